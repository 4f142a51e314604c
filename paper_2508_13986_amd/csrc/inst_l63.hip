// Instantiations of the GBEES kernels for the Lorenz '63 drift (n = 3).
#include "kernels.hpp"

namespace gbees {

const KernelTable* table_l63(int n, int precision) {
  switch (n) {
    case 3: return precision == 0 ? Ops<3, kModelL63, double>::table(0) : Ops<3, kModelL63, float>::table(1);
    default: return nullptr;
  }
}

}  // namespace gbees
