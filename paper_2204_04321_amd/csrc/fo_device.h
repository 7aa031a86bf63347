// Device helpers shared by the mesh-derived kernels (shallow-ice guess, column features).
#pragma once

#include <hip/hip_runtime.h>

#include "fo_internal.h"

namespace fo {

// Area-weighted mean over the base cells around vertex v of the cell gradient of the
// interpolated surface (triangles: P1 gradient; quads: bilinear gradient at the centre).
__device__ inline void vertex_surface_gradient(const MeshView &m, const int32_t *__restrict__ vc_ptr,
                                               const int32_t *__restrict__ vc_idx, int v, double &gx_out,
                                               double &gy_out) {
  const int nv = m.nv;
  double wsum = 0.0, gxs = 0.0, gys = 0.0;
  for (int p = vc_ptr[v]; p < vc_ptr[v + 1]; ++p) {
    const int t = vc_idx[p];
    double px[4], py[4], ps[4];
    for (int a = 0; a < nv; ++a) {
      const int w = m.cells[int64_t(t) * nv + a];
      const double4 g = m.geo[w];
      px[a] = g.x; py[a] = g.y; ps[a] = m.sb[w].x;
    }
    double gx, gy, area;
    if (nv == 3) {
      const double area2 = (px[1] - px[0]) * (py[2] - py[0]) - (px[2] - px[0]) * (py[1] - py[0]);
      gx = ((ps[1] - ps[0]) * (py[2] - py[0]) - (ps[2] - ps[0]) * (py[1] - py[0])) / area2;
      gy = ((ps[2] - ps[0]) * (px[1] - px[0]) - (ps[1] - ps[0]) * (px[2] - px[0])) / area2;
      area = 0.5 * area2;
    } else {
      const double dxi[4] = {-0.5, 0.5, 0.5, -0.5}, deta[4] = {-0.5, -0.5, 0.5, 0.5};
      double j00 = 0, j01 = 0, j10 = 0, j11 = 0, d0 = 0, d1 = 0;
      for (int a = 0; a < 4; ++a) {
        j00 += px[a] * dxi[a]; j01 += px[a] * deta[a];
        j10 += py[a] * dxi[a]; j11 += py[a] * deta[a];
        d0 += ps[a] * dxi[a];  d1 += ps[a] * deta[a];
      }
      const double det = j00 * j11 - j01 * j10;
      gx = (j11 * d0 - j10 * d1) / det;
      gy = (-j01 * d0 + j00 * d1) / det;
      double sh = 0.0;
      for (int a = 0; a < 4; ++a) sh += px[a] * py[(a + 1) & 3] - px[(a + 1) & 3] * py[a];
      area = 0.5 * fabs(sh);
    }
    wsum += area;
    gxs += area * gx;
    gys += area * gy;
  }
  gx_out = gxs / wsum;
  gy_out = gys / wsum;
}

}  // namespace fo
