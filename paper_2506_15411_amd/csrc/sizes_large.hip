// Two-level axis lengths of the lens and served-batch grids.
//   121 = 11 x 11, 189 = 27 x 7 (the 32 um lens volume of the optimisation
//   benchmark, 189 x 189 x 121 at 177 nm), 192 = 16 x 12, 256 = 16 x 16,
//   261 = 29 x 9 = 3^2 29, 275 = 25 x 11 = 5^2 11, 315 = 35 x 9 = 3^2 5 7
//   (z: 15 x 21, so the z-pass level B runs over (component, k1) threads),
//   621 = 27 x 23 = 3^3 23 (x/y only).
#include "kernels.hpp"

namespace cbs {
const SizeOps* sizes_large(int* count) {
  static const SizeOps table[] = {
    CBS_SIZE_XYZ(121, 11, 11, 11, 11), CBS_SIZE_XYZ(189, 27, 7, 27, 7),
    CBS_SIZE_XYZ(192, 16, 12, 24, 8),  CBS_SIZE_XYZ(256, 16, 16, 32, 8),
    CBS_SIZE_XYZ(261, 29, 9, 29, 9),  CBS_SIZE_XYZ(275, 25, 11, 25, 11),
    CBS_SIZE_XYZ(315, 35, 9, 15, 21), CBS_SIZE_XY(621, 27, 23)};
  *count = int(sizeof(table) / sizeof(table[0]));
  return table;
}
}  // namespace cbs
