// Ocean back-pressure on the marine margin (arXiv:2204.04321 Sec. 2, the lateral boundary
// condition on the ice margin), integrated once per mesh at upload: the load does not
// depend on the velocity, so it is memoised with the other solution-independent data
// (Sec. 4.1) and only added to the residual by the assembly kernel.
//
// Reading of the printed condition (its max(z, 0) and sign are garbled): on a marked
// front, 2 mu eps_i . n - rho g (s - z) n_i = -rho_w g max(-z, 0) n_i with sea level at
// z = 0, so the residual row (node a, component i) gains -int phi_a p n_i dA with
// p = rho g (s - z) - rho_w g max(-z, 0).
//
// A front face is the vertical quadrilateral over a boundary edge (a, b) between levels k
// and k+1.  It lies in the vertical plane of its edge, so n is the edge's horizontal
// outward normal, and with t in [0,1] along the edge and zeta in [0,1] between the levels,
// z = zl(t) + zeta dz(t) (zl, dz linear in t), dA = |edge| dz dt dzeta, and the corner
// basis functions are (1-t)(1-zeta), t(1-zeta), t zeta, (1-t) zeta.
//   * ice part rho g (s - z): degree 3 in t, 2 in zeta: 2 x 2 Gauss is exact;
//   * water part rho_w g z (z < 0): on t-intervals where the whole layer is submerged the
//     zeta integral is a polynomial (dz (zl/2 + dz/6) or dz (zl/2 + dz/3)); where the sea
//     level crosses the layer, integrating z from zl to 0 in u = zeta dz gives -zl^2/2 and
//     zl^3 / (6 dz) terms; the latter is rational in t and is integrated exactly after the
//     substitution w = dz(t) (a polynomial in w plus a logarithm), or by 16-point Gauss when
//     dz varies by less than half its size over the interval.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "fo_internal.h"

namespace fo {
namespace {

// Gauss-Legendre points and weights on [0, 1] (Newton iteration on the Legendre recurrence).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double r = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = r;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (r * p1 - p0) / (r * r - 1.0);
      const double dr = p1 / dp;
      r -= dr;
      if (std::fabs(dr) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - r);
    w[i] = 1.0 / ((1.0 - r * r) * dp * dp);
  }
}

struct Lin {   // c0 + c1 t
  double c0, c1;
  double operator()(double t) const { return c0 + c1 * t; }
};

// int_{t0}^{t1} T(t) zl(t)^3 / dz(t) dt, T = 1 - t (corner a) or t (corner b).
double rational_part(bool corner_b, const Lin &zl, const Lin &dz, double t0, double t1,
                     const std::vector<double> &gx, const std::vector<double> &gw) {
  const double e = dz.c1, d = std::min(dz(t0), dz(t1));
  if (std::fabs(e) * (t1 - t0) <= 0.5 * d) {
    double s = 0.0;
    for (size_t i = 0; i < gx.size(); ++i) {
      const double t = t0 + (t1 - t0) * gx[i];
      const double T = corner_b ? t : 1.0 - t;
      const double z = zl(t);
      s += gw[i] * T * z * z * z / dz(t);
    }
    return s * (t1 - t0);
  }
  // w = dz(t): t = (w - dz.c0) / e, zl = al + be w, T = ga + de w
  const double be = zl.c1 / e, al = zl.c0 - zl.c1 * dz.c0 / e;
  const double de = corner_b ? 1.0 / e : -1.0 / e;
  const double ga = corner_b ? -dz.c0 / e : 1.0 + dz.c0 / e;
  // (ga + de w)(al + be w)^3 = sum_m c[m] w^m
  const double a3[4] = {al * al * al, 3.0 * al * al * be, 3.0 * al * be * be, be * be * be};
  double c[5] = {0, 0, 0, 0, 0};
  for (int m = 0; m < 4; ++m) {
    c[m] += ga * a3[m];
    c[m + 1] += de * a3[m];
  }
  const double w0 = dz(t0), w1 = dz(t1);
  double s = c[0] * std::log(w1 / w0);
  double p0 = 1.0, p1 = 1.0;
  for (int m = 1; m <= 4; ++m) {
    p0 *= w0;
    p1 *= w1;
    s += c[m] * (p1 - p0) / m;
  }
  return s / e;
}

// Loads int phi p dA (without the -n factor) at the corners (a,k), (b,k), (b,k+1), (a,k+1).
void face_integral(double len, const double zc[4], double sa, double sb, double rg, double rwg,
                   const std::vector<double> &gx, const std::vector<double> &gw, double out[4]) {
  const Lin zl{zc[0], zc[1] - zc[0]}, zh{zc[3], zc[2] - zc[3]};
  const Lin dz{zh.c0 - zl.c0, zh.c1 - zl.c1}, sf{sa, sb - sa};
  static const double G[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const int Tb[4] = {0, 1, 1, 0}, Zu[4] = {0, 0, 1, 1};
  for (int c = 0; c < 4; ++c) out[c] = 0.0;
  // ice part
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const double t = G[i], zeta = G[j];
      const double z = zl(t) + zeta * dz(t);
      const double v = 0.25 * dz(t) * rg * (sf(t) - z);
      for (int c = 0; c < 4; ++c) out[c] += v * (Tb[c] ? t : 1.0 - t) * (Zu[c] ? zeta : 1.0 - zeta);
    }
  // water part, on t-intervals split where the sea level crosses the lower or upper edge
  double br[4] = {0.0, 1.0, 0.0, 0.0};
  int nb = 2;
  for (const Lin *q : {&zl, &zh}) {
    if (q->c1 != 0.0) {
      const double r = -q->c0 / q->c1;
      if (r > 0.0 && r < 1.0) br[nb++] = r;
    }
  }
  std::sort(br, br + nb);
  double wat[4] = {0, 0, 0, 0};
  for (int p = 0; p + 1 < nb; ++p) {
    const double t0 = br[p], t1 = br[p + 1];
    if (!(t1 > t0)) continue;
    const double tm = 0.5 * (t0 + t1);
    if (zl(tm) >= 0.0) continue;          // dry
    const bool whole = zh(tm) <= 0.0;     // the whole layer is under water
    for (int c = 0; c < 4; ++c) {
      double v = 0.0;
      if (whole) {
        for (int i = 0; i < 2; ++i) {
          const double t = t0 + (t1 - t0) * G[i];
          const double T = Tb[c] ? t : 1.0 - t;
          v += 0.5 * (t1 - t0) * T * dz(t) * (0.5 * zl(t) + dz(t) / (Zu[c] ? 3.0 : 6.0));
        }
      } else {
        double sq = 0.0;
        for (int i = 0; i < 2; ++i) {
          const double t = t0 + (t1 - t0) * G[i];
          const double T = Tb[c] ? t : 1.0 - t;
          sq += 0.5 * (t1 - t0) * T * zl(t) * zl(t);
        }
        const double cu = rational_part(Tb[c] != 0, zl, dz, t0, t1, gx, gw) / 6.0;
        v = Zu[c] ? cu : -0.5 * sq - cu;
      }
      wat[c] += v;
    }
  }
  for (int c = 0; c < 4; ++c) out[c] = len * (out[c] + rwg * wat[c]);
}

}  // namespace

fo_status build_front_loads(const fo_mesh_desc *d, const std::vector<double> &sig, std::vector<int32_t> &vtx,
                            std::vector<double> &load) {
  vtx.clear();
  load.clear();
  if (d->n_front_edges == 0) return FO_OK;
  if (d->n_front_edges < 0 || !d->front_edges)
    return fail(FO_EINVAL, "fo_mesh_create: front_edges is NULL or n_front_edges < 0");
  if (!(d->rho_w > 0) || !std::isfinite(d->rho_w))
    return fail(FO_EINVAL, "fo_mesh_create: rho_w must be finite and > 0 with ocean fronts");
  const int nv = d->elem == FO_HEX8 ? 4 : 3;
  const int64_t V = d->n_base_verts, T = d->n_base_cells, L = int64_t(sig.size()) - 1;
  // directed edges of the counter-clockwise cells
  std::map<std::pair<int32_t, int32_t>, int> dir;
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < nv; ++a)
      dir[{d->base_cells[t * nv + a], d->base_cells[t * nv + (a + 1) % nv]}]++;
  std::vector<std::pair<int32_t, int32_t>> edges;
  std::map<std::pair<int32_t, int32_t>, int> seen;
  for (int32_t i = 0; i < d->n_front_edges; ++i) {
    const int32_t p = d->front_edges[2 * i], q = d->front_edges[2 * i + 1];
    if (p < 0 || p >= V || q < 0 || q >= V || p == q)
      return fail(FO_EINVAL, "fo_mesh_create: front edge " + std::to_string(i) + " has a bad vertex");
    const bool fw = dir.count({p, q}) > 0, bw = dir.count({q, p}) > 0;
    if (fw && bw)
      return fail(FO_EINVAL, "fo_mesh_create: front edge " + std::to_string(i) + " is shared by two cells");
    if (!fw && !bw)
      return fail(FO_EINVAL, "fo_mesh_create: front edge " + std::to_string(i) + " is not an edge of the base mesh");
    const std::pair<int32_t, int32_t> e = fw ? std::make_pair(p, q) : std::make_pair(q, p);
    if (seen[{std::min(p, q), std::max(p, q)}]++)
      return fail(FO_EINVAL, "fo_mesh_create: front edge " + std::to_string(i) + " is listed twice");
    edges.push_back(e);
  }
  std::vector<int32_t> slot(V, -1);
  int32_t ns = 0;
  for (auto &e : edges)
    for (int32_t v : {e.first, e.second})
      if (slot[v] < 0) {
        slot[v] = ns++;
        vtx.push_back(v);
      }
  load.assign(size_t(ns) * (L + 1) * 2, 0.0);
  std::vector<double> gx, gw;
  gauss_legendre(16, gx, gw);
  const double rg = d->rho * d->g, rwg = d->rho_w * d->g;
  for (auto &e : edges) {
    const int32_t a = e.first, b = e.second;
    const double dx = d->base_xy[2 * b] - d->base_xy[2 * a], dy = d->base_xy[2 * b + 1] - d->base_xy[2 * a + 1];
    const double len = std::hypot(dx, dy);
    const double nx = dy / len, ny = -dx / len;   // the cell lies to the left of a -> b
    const double ba = d->surface[a] - d->thickness[a], bb = d->surface[b] - d->thickness[b];
    for (int64_t k = 0; k < L; ++k) {
      const double zc[4] = {ba + sig[k] * d->thickness[a], bb + sig[k] * d->thickness[b],
                            bb + sig[k + 1] * d->thickness[b], ba + sig[k + 1] * d->thickness[a]};
      double f[4];
      face_integral(len, zc, d->surface[a], d->surface[b], rg, rwg, gx, gw, f);
      const int32_t vtx[4] = {a, b, b, a};
      const int64_t lev[4] = {k, k, k + 1, k + 1};
      for (int c = 0; c < 4; ++c) {
        double *dst = load.data() + (size_t(slot[vtx[c]]) * (L + 1) + lev[c]) * 2;
        dst[0] -= f[c] * nx;
        dst[1] -= f[c] * ny;
      }
    }
  }
  return FO_OK;
}

}  // namespace fo
