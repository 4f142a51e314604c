// Instantiations of the GBEES kernels for the linear test drift, n = 1..3.
#include "kernels.hpp"

namespace gbees {

const KernelTable* table_linear_a(int n, int precision) {
  switch (n) {
    case 1: return precision == 0 ? Ops<1, kModelLinear, double>::table(0) : Ops<1, kModelLinear, float>::table(1);
    case 2: return precision == 0 ? Ops<2, kModelLinear, double>::table(0) : Ops<2, kModelLinear, float>::table(1);
    case 3: return precision == 0 ? Ops<3, kModelLinear, double>::table(0) : Ops<3, kModelLinear, float>::table(1);
    default: return nullptr;
  }
}

}  // namespace gbees
