// Instantiations of the GBEES kernels for the linear test drift, n = 4..6.
#include "kernels.hpp"

namespace gbees {

const KernelTable* table_linear_b(int n, int precision) {
  switch (n) {
    case 4: return precision == 0 ? Ops<4, kModelLinear, double>::table(0) : Ops<4, kModelLinear, float>::table(1);
    case 5: return precision == 0 ? Ops<5, kModelLinear, double>::table(0) : Ops<5, kModelLinear, float>::table(1);
    case 6: return precision == 0 ? Ops<6, kModelLinear, double>::table(0) : Ops<6, kModelLinear, float>::table(1);
    default: return nullptr;
  }
}

}  // namespace gbees
