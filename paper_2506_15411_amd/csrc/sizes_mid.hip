// Two-level axis lengths 36..128: (n1, n2) for the x/y passes, (z1, z2) for
// the z pass (z2 small: a z-pass thread holds 3 * z2 complex values).
#include "kernels.hpp"

namespace cbs {
const SizeOps* sizes_mid(int* count) {
  static const SizeOps table[] = {
    CBS_SIZE_XYZ(36, 6, 6, 9, 4),     CBS_SIZE_XYZ(40, 8, 5, 8, 5),
    CBS_SIZE_XYZ(48, 8, 6, 16, 3),    CBS_SIZE_XYZ(64, 8, 8, 16, 4),
    CBS_SIZE_XYZ(96, 12, 8, 24, 4),   CBS_SIZE_XYZ(100, 10, 10, 25, 4),
    CBS_SIZE_XYZ(128, 16, 8, 32, 4)};
  *count = int(sizeof(table) / sizeof(table[0]));
  return table;
}
}  // namespace cbs
