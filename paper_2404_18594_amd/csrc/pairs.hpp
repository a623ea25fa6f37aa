// Site pairs of the correlation classes of the observables: displacement
// (|dx|, |dy|) = (1,0), (0,1), (1,1), (2,0), (0,2), minimum image on
// periodic sides (Sec. III definition of C^sp, summed over ordered pairs).
#pragma once

#include "common.hpp"

namespace cdtwa {

__device__ inline int min_image(int dd, int L, int periodic) {
  if (!periodic) return dd < 0 ? -dd : dd;
  int m = ((dd % L) + L) % L;
  return (L - m < m) ? L - m : m;
}

// f(j, cls) for every site j != i whose displacement from i falls in class
// cls, each such j once (small periodic sides fold displacements together)
template <typename F>
__device__ inline void for_each_class_pair(const Geom& g, int i, F&& f) {
  const int dxs[12] = {1, -1, 0, 0, 1, 1, -1, -1, 2, -2, 0, 0};
  const int dys[12] = {0, 0, 1, -1, 1, -1, 1, -1, 0, 0, 2, -2};
  const int cdx[5] = {1, 0, 1, 2, 0}, cdy[5] = {0, 1, 1, 0, 2};
  const int xi = i % g.Lx, yi = i / g.Lx;
  int seen[12];
  int nseen = 0;
  for (int v = 0; v < 12; ++v) {
    int xj = xi + dxs[v], yj = yi + dys[v];
    if (g.periodic) {
      xj = ((xj % g.Lx) + g.Lx) % g.Lx;
      yj = ((yj % g.Ly) + g.Ly) % g.Ly;
    } else if (xj < 0 || xj >= g.Lx || yj < 0 || yj >= g.Ly) {
      continue;
    }
    const int j = yj * g.Lx + xj;
    if (j == i) continue;
    bool dup = false;
    for (int s = 0; s < nseen; ++s) dup |= (seen[s] == j);
    if (dup) continue;
    seen[nseen++] = j;
    const int ax = min_image(xj - xi, g.Lx, g.periodic), ay = min_image(yj - yi, g.Ly, g.periodic);
    int cls = -1;
    for (int c = 0; c < 5; ++c)
      if (ax == cdx[c] && ay == cdy[c]) cls = c;
    if (cls >= 0) f(j, cls);
  }
}

}  // namespace cdtwa
