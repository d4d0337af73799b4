// pkh_tiles.h -- the tile shapes the stage kernels are compiled for and the
// host-side choice among them (plain C++, also built for the host tests).
#pragma once

#include <stdint.h>

namespace pkh {

// Rows per workgroup tile for a block of n1 x n2 cells and a requested value
// tj (0: default) of a stage with piecewise-linear (recon 1) or donor-cell
// (recon 0) faces; -1 if no compiled variant fits.
//
// Compiled (n1, rows) variants, the default first: n1 = 8: 8; n1 = 16: 8,
// 16, 4; n1 = 32: 8, 4, 16; n1 = 64: 4, 2. An explicit request must be one
// of them and divide n2. Defaults: on 32-cell rows both stages take 8 rows
// (256 threads, three waves per SIMD); on 16-cell rows both take 16 rows
// from 1024 waves on, else 8 (nblocks, the blocks of the launch, 0 when
// unknown). Measured at 256^3 on line-aligned state rows: on 32-cell rows
// the corrector 0.69-0.71 ms on 8 rows against 0.74 ms on 16 and 0.81 ms on
// 4, the predictor 0.400 ms on 8 rows against 0.412-0.430 ms on 16; on
// 16-cell rows 16 rows against 8 save 5 % of the cycle. When the preferred
// default does not divide n2 the default is the largest compiled variant
// below it that does (then the largest that does at all).
inline int stage_tile_rows(int n1, int n2, int tj, int64_t nblocks = 0, int recon = 1) {
  static const int opts[4][3] = {{8, 0, 0}, {8, 16, 4}, {8, 4, 16}, {4, 2, 0}};
  const int row = n1 == 8 ? 0 : n1 == 16 ? 1 : n1 == 32 ? 2 : n1 == 64 ? 3 : -1;
  if (row < 0 || n2 <= 0) return -1;
  if (tj != 0) {
    for (int q = 0; q < 3; ++q)
      if (opts[row][q] == tj && tj > 0 && n2 % tj == 0) return tj;
    return -1;
  }
  int want = opts[row][0];
  const int64_t waves = nblocks * n1 * n2 / 64;
  if (n1 == 16 && nblocks > 0 && waves >= 1024) want = 16;
  int best = -1, any = -1;
  for (int q = 0; q < 3; ++q) {
    const int o = opts[row][q];
    if (o <= 0 || n2 % o) continue;
    if (o <= want && o > best) best = o;
    if (o > any) any = o;
  }
  return best > 0 ? best : any;
}

}  // namespace pkh
