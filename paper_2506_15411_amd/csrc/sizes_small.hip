// Axis lengths 2..32 handled by a single register codelet (n = n x 1).
#include "kernels.hpp"

namespace cbs {
#define S1(n) CBS_SIZE_XYZ(n, n, 1, n, 1)
const SizeOps* sizes_small(int* count) {
  static const SizeOps table[] = {
    S1(2),  S1(3),  S1(4),  S1(5),  S1(6),  S1(7),  S1(8),  S1(9),  S1(10), S1(11), S1(12),
    S1(13), S1(14), S1(15), S1(16), S1(18), S1(20), S1(24), S1(25), S1(27), S1(29), S1(32)};
  *count = int(sizeof(table) / sizeof(table[0]));
  return table;
}
}  // namespace cbs
