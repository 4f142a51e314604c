// Instantiations of the GBEES kernels for the Lorenz '96 drift (n = 4..6).
#include "kernels.hpp"

namespace gbees {

const KernelTable* table_l96(int n, int precision) {
  switch (n) {
    case 4: return precision == 0 ? Ops<4, kModelL96, double>::table(0) : Ops<4, kModelL96, float>::table(1);
    case 5: return precision == 0 ? Ops<5, kModelL96, double>::table(0) : Ops<5, kModelL96, float>::table(1);
    case 6: return precision == 0 ? Ops<6, kModelL96, double>::table(0) : Ops<6, kModelL96, float>::table(1);
    default: return nullptr;
  }
}

}  // namespace gbees
