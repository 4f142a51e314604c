// Selects the kernel instantiation of a (model, dimension, precision) triple.
#include "gbees_host.hpp"

namespace gbees {

const KernelTable* table_l63(int n, int precision);
const KernelTable* table_l96(int n, int precision);
const KernelTable* table_linear_a(int n, int precision);
const KernelTable* table_linear_b(int n, int precision);

const KernelTable* kernel_table(int model, int n, int precision) {
  if (precision != 0 && precision != 1) return nullptr;
  if (model == kModelL63) return table_l63(n, precision);
  if (model == kModelL96) return table_l96(n, precision);
  if (model == kModelLinear) return n <= 3 ? table_linear_a(n, precision) : table_linear_b(n, precision);
  return nullptr;
}

}  // namespace gbees
