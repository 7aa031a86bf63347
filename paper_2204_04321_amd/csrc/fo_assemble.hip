// Cell-parallel assembly of the first-order Stokes residual and Jacobian on gfx950.
//
// Physics (arXiv:2204.04321 Sec. 2): momentum balance eq. (FOStokes) with the
// strain-rate vectors eps1 = (2 e_xx + e_yy, e_xy, e_xz), eps2 = (e_xy,
// e_xx + 2 e_yy, e_yz); Glen viscosity eq. (effvisc) with the effective strain
// rate eq. (effeps), regularised by eps0; stress-free surface; linear bed
// friction beta u.  Discrete residual eq. (residual); Jacobian eq. (linearsystem)
// by forward-mode AD (Sec. 3.2): the tangent of the element residual along each
// element dof is pushed through strain rate -> eps_e^2 -> mu -> residual.
//
// Owner-computes decomposition.  Every CSR row block belongs to one vertex column
// v (all dofs of v, every level).  Work item = (v, base cell t around v): one lane
// walks the column of t from the bed up, layer by layer, and evaluates each cell
// at its quadrature points (geometry, strain rate, viscosity: the primal), then
// the residual rows of v's two nodes in the cell and their derivatives along all
// element dofs (the AD tangents, one register accumulator per derivative
// direction and row).  A wave owns a run of consecutive vertex columns (<= 64
// items); its lanes add their rows into a two-level window of those columns in
// LDS, and once level k has received both cells that touch it (layers k-1 and k)
// the wave copies it into its contiguous CSR range.  No global atomics, no
// zero fill of J or R, every value written once; results do not depend on
// scheduling.  Each cell is evaluated by each of its vertex columns (3 or 4
// times) in exchange.
//
// Wedge kernels run two waves per SIMD (256 registers per lane, a few per-layer spills).
// Their tangents are accumulated in factorised form (per row node and component pair:
// two weighted sums of the row coefficients and one projection per triangle point), and
// the twelve column blocks are formed once per layer; the level windows are FP64 for
// either Jacobian value type.
//
// CSR slot of row (v, level kr, comp c) and column (vertex of rank r in v's sorted
// neighbour list, level kc, comp d): colptr[v] + 4 D_v cumlev(kr) + c 2 nlev(kr) D_v
// + r 2 nlev(kr) + 2 (kc - max(kr-1, 0)) + d.
#include <hip/hip_runtime.h>

#include "fo_internal.h"

// Multiply-adds are fused only where one source expression holds both operations, so
// the residual-only, R+J and ensemble kernels, which share the element arithmetic, round
// it identically (fusion chosen by the backend depends on each kernel's other uses).
#pragma clang fp contract(on)

namespace fo {
namespace {

constexpr int WAVE = 64;

constexpr double G1 = 0.21132486540518711775;   // 1/2 - 1/(2 sqrt 3)
constexpr double G2 = 0.78867513459481288225;   // 1/2 + 1/(2 sqrt 3)

template <int NV>
struct Elem;
template <>
struct Elem<3> {  // wedge: P1 triangle x linear in zeta
  static constexpr int NPE = 6, NQ = 6, NQB = 3;
};
template <>
struct Elem<4> {  // hexahedron: bilinear quad x linear in zeta
  static constexpr int NPE = 8, NQ = 8, NQB = 4;
};

// Quadrature on the reference cell ([0,1]^2 or the unit triangle, zeta in [0,1]):
// weights, zeta, 2D basis values and reference derivatives at each point.
struct QTable {
  double w[8], zeta[8], lam[8][4], dlx[8][4], dly[8][4];
  double bw[4], blam[4][4], bdlx[4][4], bdly[4][4];
};

__constant__ QTable kQ[2];   // [0] wedge, [1] hex

constexpr void basis2d_tab(int nv, double xi, double eta, double *lam, double *dx, double *dy) {
  if (nv == 3) {
    lam[0] = 1.0 - xi - eta; lam[1] = xi; lam[2] = eta; lam[3] = 0.0;
    dx[0] = -1.0; dx[1] = 1.0; dx[2] = 0.0; dx[3] = 0.0;
    dy[0] = -1.0; dy[1] = 0.0; dy[2] = 1.0; dy[3] = 0.0;
  } else {
    const double mx = 1.0 - xi, my = 1.0 - eta;
    lam[0] = mx * my; lam[1] = xi * my; lam[2] = xi * eta; lam[3] = mx * eta;
    dx[0] = -my; dx[1] = my; dx[2] = eta; dx[3] = -eta;
    dy[0] = -mx; dy[1] = -xi; dy[2] = xi; dy[3] = mx;
  }
}

constexpr QTable make_table(int nv) {
  QTable t{};
  const int nq = nv == 3 ? 6 : 8, nqb = nv == 3 ? 3 : 4;
  for (int q = 0; q < nq; ++q) {
    double xi = 0, eta = 0, zeta = 0, w = 0;
    if (nv == 3) {
      const int tq = q % 3;
      xi = (tq == 1) ? 2.0 / 3.0 : 1.0 / 6.0;
      eta = (tq == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
      zeta = (q < 3) ? G1 : G2;
      w = 1.0 / 12.0;
    } else {
      xi = (q & 1) ? G2 : G1;
      eta = (q & 2) ? G2 : G1;
      zeta = (q & 4) ? G2 : G1;
      w = 0.125;
    }
    t.w[q] = w;
    t.zeta[q] = zeta;
    basis2d_tab(nv, xi, eta, t.lam[q], t.dlx[q], t.dly[q]);
  }
  for (int r = 0; r < nqb; ++r) {
    double xi = 0, eta = 0;
    if (nv == 3) {
      xi = (r == 1) ? 2.0 / 3.0 : 1.0 / 6.0;
      eta = (r == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
      t.bw[r] = 1.0 / 6.0;
    } else {
      xi = (r & 1) ? G2 : G1;
      eta = (r & 2) ? G2 : G1;
      t.bw[r] = 0.25;
    }
    basis2d_tab(nv, xi, eta, t.blam[r], t.bdlx[r], t.bdly[r]);
  }
  return t;
}

__device__ __forceinline__ int nlev(int k, int L) { return (k == 0 || k == L) ? 2 : 3; }
__device__ __forceinline__ int cumlev(int k) { return k == 0 ? 0 : 3 * k - 1; }

// 1/x: hardware estimate refined by two Newton steps (full double precision).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// x^(-1/3) for x > 0: single-precision exp2/log2 estimate (~1e-7) refined by two Newton
// steps on y^-3 = x, y <- y (4 - x y^3) / 3 (quadratic convergence to double precision).
__device__ __forceinline__ double rcbrt64(double x) {
  const double y = double(__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(float(x)) * (1.0f / 3.0f)));
  // one third-order step: with r = 1 - x y^3, x^(-1/3) = y (1 - r)^(-1/3)
  // = y (1 + r/3 + 2 r^2/9 + O(r^3)), and |r| ~ 1e-7 leaves O(1e-21)
  const double r = fma(-x, y * y * y, 1.0);
  return fma(y * r, fma(2.0 / 9.0, r, 1.0 / 3.0), y);
}

// q^p for the viscosity power, q = eps_e^2 + eps0^2 >= 0: exp2(p log2 q), which needs none
// of the general pow's cases for negative or special arguments; p = 0 (n = 1) gives 1.
__device__ __forceinline__ double powq(double q, double p) {
  return p == 0.0 ? 1.0 : exp2(p * log2(q));
}

template <class T>
__device__ __forceinline__ void lds_add(T *p, T v) {
  atomicAdd(p, v);   // LDS atomics: lanes of one wave may hit the same entry
}

// The block is one wave: a workgroup barrier orders its LDS traffic.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Picks a, b, c or d by a lane-varying index i (d for any i outside 0..2) without a branch:
// all four operands are evaluated and combined through bit masks.  Written as a compare
// chain, the selection becomes a switch, i.e. a divergent branch tree, and the register
// allocator has placed copies of values that stay live across it inside the masked part,
// so lanes outside the mask later read copies they never wrote.
__device__ __forceinline__ double sel4(int i, double a, double b, double c, double d) {
  using u64 = unsigned long long;
  const u64 m0 = 0ull - u64(i == 0), m1 = 0ull - u64(i == 1), m2 = 0ull - u64(i == 2);
  const u64 m3 = ~(m0 | m1 | m2);
  const u64 r = (__builtin_bit_cast(u64, a) & m0) | (__builtin_bit_cast(u64, b) & m1) |
                (__builtin_bit_cast(u64, c) & m2) | (__builtin_bit_cast(u64, d) & m3);
  return __builtin_bit_cast(double, r);
}

// Two consecutive Jacobian entries as one streaming (nontemporal) store; p is 8-entry aligned.
template <class JT>
__device__ __forceinline__ void store2_nt(JT *p, double x, double y) {
  typedef JT v2 __attribute__((ext_vector_type(2)));
  v2 t;
  t.x = JT(x);
  t.y = JT(y);
  __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(p));
}

// Tetrahedral extrusion: one layer of a base triangle's prism, split into three
// tetrahedra by the global order of its corners (the corners arrive sorted, so corner r
// has the r-th smallest vertex id): (0,1,2,0'), (1,2,0',1'), (2,0',1',2'), primes one level
// up.  Linear basis: gradients, strain rate and viscosity are constant on a tetrahedron,
// so every integral is exact (V times the integrand, int phi_a = V/4).  Adds the residual
// rows of the item's two nodes (corner ra at the lower and upper level) and their
// derivatives along the prism's 12 dofs: Jx[row level][c][d][corner][level].
constexpr int TET_R[3][4] = {{0, 1, 2, 0}, {1, 2, 0, 1}, {2, 0, 1, 2}};   // corner of node a
constexpr int TET_L[3][4] = {{0, 0, 0, 1}, {0, 0, 1, 1}, {0, 1, 1, 1}};   // level of node a

template <class AT, bool JAC, bool N3>
__device__ __forceinline__ void tet_layer(const MeshView &m, int ra, int picard, const double *xr, const double *yr,
                                          const double *zlo, const double *dz, const double *ulo,
                                          const double *du, const double *vlo, const double *dv,
                                          const double *sv, double &Rb0, double &Rb1, double &Rt0, double &Rt1,
                                          AT (&Jx)[2][2][2][3][2]) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double X[4][3], ua[4], va[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = TET_R[q][a], l = TET_L[q][a];
      X[a][0] = xr[r];
      X[a][1] = yr[r];
      X[a][2] = l ? zlo[r] + dz[r] : zlo[r];
      ua[a] = l ? ulo[r] + du[r] : ulo[r];
      va[a] = l ? vlo[r] + dv[r] : vlo[r];
    }
    // rows of M: edges from node 0; columns of M^-1 are the gradients of phi_1..3
    double e[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) e[j][i] = X[j + 1][i] - X[0][i];
    double cr[3][3];   // cr[j] = e[j+1] x e[j+2]
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double *p = e[(j + 1) % 3], *w = e[(j + 2) % 3];
      cr[j][0] = p[1] * w[2] - p[2] * w[1];
      cr[j][1] = p[2] * w[0] - p[0] * w[2];
      cr[j][2] = p[0] * w[1] - p[1] * w[0];
    }
    const double det = e[0][0] * cr[0][0] + e[0][1] * cr[0][1] + e[0][2] * cr[0][2];
    const double idet = rcp64(det);
    double g[4][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      g[1][i] = cr[0][i] * idet;
      g[2][i] = cr[1][i] * idet;
      g[3][i] = cr[2][i] * idet;
      g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
    }
    const double V = fabs(det) * (1.0 / 6.0);
    double ux = 0, uy = 0, uz = 0, vx = 0, vy = 0, vz = 0, sx = 0, sy = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ux = fma(ua[a], g[a][0], ux); uy = fma(ua[a], g[a][1], uy); uz = fma(ua[a], g[a][2], uz);
      vx = fma(va[a], g[a][0], vx); vy = fma(va[a], g[a][1], vy); vz = fma(va[a], g[a][2], vz);
      sx = fma(sv[TET_R[q][a]], g[a][0], sx); sy = fma(sv[TET_R[q][a]], g[a][1], sy);
    }
    const double exx = ux, eyy = vy, exy = 0.5 * (uy + vx), exz = 0.5 * uz, eyz = 0.5 * vz;
    const double qq = exx * exx + eyy * eyy + exx * eyy + exy * exy + exz * exz + eyz * eyz;
    const double qe = qq + m.eps0_sq;
    double mu;
    if constexpr (N3) mu = m.visc_pref * rcbrt64(qe);
    else mu = m.visc_pref * powq(qe, m.visc_exp);
    const double s2 = 2.0 * mu * V;
    const double t2 = picard ? 0.0 : 2.0 * (m.visc_exp * mu * rcp64(qe)) * V;
    const double E[2][3] = {{2.0 * exx + eyy, exy, exz}, {exy, exx + 2.0 * eyy, eyz}};
    const double gq = 0.25 * V * m.rho_g;       // rho g int phi_a / (d s)
    // the item's two nodes: gradient on this tetrahedron (zero if not one of its nodes)
    double gr[2][3] = {{0, 0, 0}, {0, 0, 0}}, in[2] = {0, 0};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double hit = TET_R[q][a] == ra ? 1.0 : 0.0;
      const int l = TET_L[q][a];
      in[l] += hit;
#pragma unroll
      for (int i = 0; i < 3; ++i) gr[l][i] = fma(hit, g[a][i], gr[l][i]);
    }
    double Rr[2][2];
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        Rr[l][c] = fma(s2, E[c][0] * gr[l][0] + E[c][1] * gr[l][1] + E[c][2] * gr[l][2],
                       gq * in[l] * (c ? sy : sx));
    Rb0 += Rr[0][0]; Rb1 += Rr[0][1];
    Rt0 += Rr[1][0]; Rt1 += Rr[1][1];
    if constexpr (JAC) {
      const AT s2a = AT(s2), t2a = AT(t2);
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        const AT ax = AT(gr[l][0]), ay = AT(gr[l][1]), az = AT(gr[l][2]);
        const AT Ax = s2a * ax, Ay = s2a * ay, Az = s2a * az;
        const AT T0 = t2a * AT(E[0][0] * gr[l][0] + E[0][1] * gr[l][1] + E[0][2] * gr[l][2]);
        const AT T1 = t2a * AT(E[1][0] * gr[l][0] + E[1][1] * gr[l][1] + E[1][2] * gr[l][2]);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int r = TET_R[q][b], lb = TET_L[q][b];
          const AT bx = AT(g[b][0]), by = AT(g[b][1]), bz = AT(g[b][2]);
          const AT Gu = AT(E[0][0]) * bx + AT(E[0][1]) * by + AT(E[0][2]) * bz;   // d(eps_e^2)/dU_(b,u)
          const AT Gv = AT(E[1][0]) * bx + AT(E[1][1]) * by + AT(E[1][2]) * bz;   // d(eps_e^2)/dU_(b,v)
          AT &uu = Jx[l][0][0][r][lb], &uv = Jx[l][0][1][r][lb];
          AT &vu = Jx[l][1][0][r][lb], &vv = Jx[l][1][1][r][lb];
          // K_uu = 2 ax bx + 1/2 ay by + 1/2 az bz, K_uv = ax by + 1/2 ay bx,
          // K_vu = ay bx + 1/2 ax by, K_vv = 1/2 ax bx + 2 ay by + 1/2 az bz
          uu = fma(Ax + Ax, bx, uu); uu = fma(AT(0.5) * Ay, by, uu); uu = fma(AT(0.5) * Az, bz, uu);
          uu = fma(T0, Gu, uu);
          uv = fma(Ax, by, uv); uv = fma(AT(0.5) * Ay, bx, uv); uv = fma(T0, Gv, uv);
          vu = fma(Ay, bx, vu); vu = fma(AT(0.5) * Ax, by, vu); vu = fma(T1, Gu, vu);
          vv = fma(AT(0.5) * Ax, bx, vv); vv = fma(Ay + Ay, by, vv); vv = fma(AT(0.5) * Az, bz, vv);
          vv = fma(T1, Gv, vv);
        }
      }
    }
  }
}

// One wave = one task (a run of vertex columns); one lane = one (v, t) item.
// N3 selects the n = 3 viscosity power; JAC adds the Jacobian; JT is its value type
// (double, or float with FP32 derivative arithmetic over the FP64 primal).
template <int NV, bool JAC, class JT, bool N3, bool TET = false>
__device__ __forceinline__ void owner_task(const MeshView &m, const int4 task, const double *__restrict__ U,
                                           double *__restrict__ R, JT *__restrict__ J, int picard,
                                           int max_slot, int max_tv, unsigned char *smem) {
  constexpr int NQ = Elem<NV>::NQ, NQB = Elem<NV>::NQB;
  using AT = JT;   // derivative arithmetic type
  const QTable &Q = kQ[NV == 3 ? 0 : 1];
  // The level windows accumulate in FP64 for either value type: FP32 LDS atomics on this
  // scatter pattern saturate the LDS data path (measured), FP64 ones do not.
  double *Jw = reinterpret_cast<double *>(smem);                                               // [2][max_slot]
  double *Rw = reinterpret_cast<double *>(smem + (JAC ? 2 * size_t(max_slot) * sizeof(double) : 0));  // [2][2 max_tv]
  const int lane = threadIdx.x;
  const int vb = task.y, ve = task.z, ib = task.w;
  const int ie = m.vc_ptr[ve];
  const bool act = ib + lane < ie;
  const int item = act ? ib + lane : ib;
  const int L = m.L;
  const int v = act ? m.item_vtx[item] : vb;
  const int t = act ? m.vc_idx[item] : 0;
  const int al = act ? m.vc_pos[item] : 0;
  // Prisms take their cell's corners in cyclic order starting at the item's own vertex, so
  // that vertex is always corner 0 (a cyclic rotation keeps the triangle's orientation, and
  // the triangle rules are invariant under it): its selections become constants and its
  // Jacobian entries can be carried from layer to layer in registers (below).
  constexpr bool ROT = NV == 3 && !TET;
  const int rot = ROT ? al : 0;
  const int al_own = ROT ? 0 : al;
  const int Dv = m.deg[v];
  const int soff = m.slot_off[v];
  // per-item integers fixed over the layers, packed: slot offset (12 bits, < 2048), degree
  // (8), column position in the task (6, a task has at most 64 columns), corner (2).  Each
  // layer re-derives them, the corner ranks and the corners' addresses from this word, the
  // rank word and the vertex ids, passed through an empty asm statement: otherwise the
  // compiler hoists the derived addresses out of the layer loop and spills them, and every
  // reload costs a scratch round trip that serialises the layer's gather loads.
  const uint32_t imeta_base = uint32_t(soff) | (uint32_t(Dv) << 12) | (uint32_t(v - vb) << 20);
  const uint32_t imeta_cell = imeta_base | (uint32_t(al_own) << 26);
  const int slot_size = m.slot_off[ve - 1] + 12 * m.deg[ve - 1];
  // 8 bits per corner: its rank in v's neighbour list
  uint32_t irank = act ? m.item_rank[item] : 0u;
  if constexpr (ROT) irank = ((irank >> (8 * rot)) | (irank << (8 * (3 - rot)))) & 0xFFFFFFu;

  // ---- per-item constants -----------------------------------------------------------------
  int vid[NV];
  double xl[NV], yl[NV], bed[NV], Hh[NV], su[NV];
  // horizontal coordinates relative to the cell's first corner, the bed, H and s
  auto load_geo = [&](double *xl_, double *yl_, double *bed_, double *H_, double *s_) {
    double x0 = 0, y0 = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double4 g = m.geo[vid[i]];
      if (i == 0) { x0 = g.x; y0 = g.y; }
      xl_[i] = g.x - x0;
      yl_[i] = g.y - y0;
      bed_[i] = g.z;
      H_[i] = g.w;
      s_[i] = m.sb[vid[i]].x;
    }
  };
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int ci = ROT ? (i + rot >= 3 ? i + rot - 3 : i + rot) : i;
    vid[i] = m.cells[int64_t(t) * NV + ci];
  }
  load_geo(xl, yl, bed, Hh, su);
  // The layer loop walks the corners in lvid order with their neighbour ranks in lrank and
  // the item's corner al_loop: the cell's own order, or for tetrahedra the order of the
  // vertex ids (which fixes the split of each prism).
  int lvid[NV];
  uint32_t lrank = irank, imeta = imeta_cell;
#pragma unroll
  for (int i = 0; i < NV; ++i) lvid[i] = vid[i];
  if constexpr (TET) {
    int rk_of[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) rk_of[i] = int(vid[i] > vid[(i + 1) % 3]) + int(vid[i] > vid[(i + 2) % 3]);
    lrank = 0u;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      int vr = 0;
      uint32_t br = 0u;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int hit = int(rk_of[i] == r);
        vr += hit * vid[i];
        br += uint32_t(hit) * ((irank >> (8 * i)) & 255u);
      }
      lvid[r] = vr;
      lrank |= br << (8 * r);
    }
    // lanes without an item take corner 3, which no tetrahedron node has: their rows get
    // exact zeros, so the layer loop's adds need no divergent branch (see below)
    const int al_loop = act ? rk_of[0] * int(al == 0) + rk_of[1] * int(al == 1) + rk_of[2] * int(al == 2) : 3;
    imeta = imeta_base | (uint32_t(al_loop) << 26);
  }
  // P1 triangles: the horizontal basis gradients and the map determinant are constant
  double lxc[NV], lyc[NV], detc = 0, sxc = 0, syc = 0;
  if constexpr (NV == 3) {
    const double x_xi = xl[1] - xl[0], x_eta = xl[2] - xl[0];
    const double y_xi = yl[1] - yl[0], y_eta = yl[2] - yl[0];
    detc = x_xi * y_eta - x_eta * y_xi;
    const double iG = rcp64(detc);
    lxc[1] = y_eta * iG; lxc[2] = -y_xi * iG; lxc[0] = -(lxc[1] + lxc[2]);
    lyc[1] = -x_eta * iG; lyc[2] = x_xi * iG; lyc[0] = -(lyc[1] + lyc[2]);
#pragma unroll
    for (int i = 0; i < NV; ++i) { sxc += su[i] * lxc[i]; syc += su[i] * lyc[i]; }
  }
  double lx_al = 0.0, ly_al = 0.0;
  if constexpr (NV == 3) {
    lx_al = ROT ? lxc[0] : sel4(al, lxc[0], lxc[1], lxc[2], 0.0);
    ly_al = ROT ? lyc[0] : sel4(al, lyc[0], lyc[1], lyc[2], 0.0);
  }

  // metadata of the task's vertex columns, one per lane (a task has at most 64 columns)
  const int nvt = ve - vb;
  int my_deg = 0, my_soff = 0, my_col_lo = 0, my_col_hi = 0;
  if (lane < nvt) {
    my_deg = m.deg[vb + lane];
    my_soff = m.slot_off[vb + lane];
    const int64_t c = m.colptr[vb + lane];
    my_col_lo = int(uint32_t(uint64_t(c)));
    my_col_hi = int(uint32_t(uint64_t(c) >> 32));
  }

  // ---- zero both level windows -------------------------------------------------------------
  if constexpr (JAC) {
    for (int e = lane; e < slot_size; e += WAVE) { Jw[e] = 0.0; Jw[max_slot + e] = 0.0; }
  }
  for (int e = lane; e < 2 * (ve - vb); e += WAVE) { Rw[e] = 0.0; Rw[2 * max_tv + e] = 0.0; }
  wave_sync();

  // ---- bed friction on the lower face of the bottom layer: rows of v's level-0 node, added
  // to the level-0 windows before the layer loop ----------------------------------------------
  if (act) {
    double bx_[NV], by_[NV], bb_[NV], bH_[NV], bs_[NV], be[NV], zb[NV], ub[NV], vb_[NV];
    load_geo(bx_, by_, bb_, bH_, bs_);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      be[i] = m.sb[vid[i]].y;
      zb[i] = bb_[i] + m.sigma[0] * bH_[i];
      const double2 a0 = *reinterpret_cast<const double2 *>(U + 2 * (int64_t(vid[i]) * (L + 1)));
      ub[i] = a0.x; vb_[i] = a0.y;
    }
    double Rf0 = 0, Rf1 = 0;
    AT Jf[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) Jf[j] = AT(0);
#pragma unroll
    for (int r = 0; r < NQB; ++r) {
      double txx = 0, txy = 0, txz = 0, tyx = 0, tyy = 0, tyz = 0, br = 0, ur = 0, vr = 0;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const double dx = Q.bdlx[r][i], dy = Q.bdly[r][i], lm = Q.blam[r][i];
        txx += bx_[i] * dx; txy += by_[i] * dx; txz += zb[i] * dx;
        tyx += bx_[i] * dy; tyy += by_[i] * dy; tyz += zb[i] * dy;
        br += be[i] * lm; ur += ub[i] * lm; vr += vb_[i] * lm;
      }
      const double nx = txy * tyz - txz * tyy, ny = txz * tyx - txx * tyz, nz = txx * tyy - txy * tyx;
      const double wb = Q.bw[r] * sqrt(nx * nx + ny * ny + nz * nz) * br;
      const double la = ROT ? Q.blam[r][0] : sel4(al, Q.blam[r][0], Q.blam[r][1], Q.blam[r][2], Q.blam[r][NV - 1]);
      Rf0 += wb * ur * la;
      Rf1 += wb * vr * la;
#pragma unroll
      for (int j = 0; j < NV; ++j) Jf[j] += AT(wb * la * Q.blam[r][j]);
    }
    const int rl0 = 2 * (v - vb);
    lds_add(Rw + rl0, Rf0);
    lds_add(Rw + rl0 + 1, Rf1);
    if constexpr (JAC) {
      // row (v, 0, c), column (corner j, level 0, component c)
      const int nl0 = nlev(0, L);
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < NV; ++j)
          lds_add(Jw + soff + c * 2 * nl0 * Dv + int((irank >> (8 * j)) & 255u) * 2 * nl0 + c, double(Jf[j]));
    }
  }

  // FP32 tangents: the upper row's entries at the upper level of layer k are kept in
  // registers and added together with layer k + 1's lower-row entries at the same places,
  // a quarter fewer LDS adds.  The FP64 kernel has no registers to spare for them (spills
  // made it slower); on prisms it carries the four of the item's own vertex (corner 0),
  // which every item of a vertex adds to the same window places, in a per-lane LDS slot
  // after the residual windows (registers spilled them to scratch every layer).
  constexpr bool CARRY = JAC && sizeof(JT) == 4;
  constexpr bool CARRY0 = JAC && ROT && !CARRY;
  AT carry[2][2][NV];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int j = 0; j < NV; ++j) carry[c][d][j] = AT(0);
  double *carry0 = Rw + 4 * size_t(max_tv) + 4 * lane;   // [c][d] of this lane

  for (int k = 0; k < L; ++k) {
    const int cur = k & 1, nxt = cur ^ 1;
    uint32_t ipy = lrank, imt = imeta;
    int vidk[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vidk[i] = lvid[i];
    // one statement, so that reloads of spilled operands are issued together
    if constexpr (NV == 3)
      asm volatile("" : "+v"(ipy), "+v"(imt), "+v"(vidk[0]), "+v"(vidk[1]), "+v"(vidk[2]));
    else
      asm volatile("" : "+v"(ipy), "+v"(imt), "+v"(vidk[0]), "+v"(vidk[1]), "+v"(vidk[2]), "+v"(vidk[NV - 1]));
    const int al = int(imt >> 26), soff = int(imt & 4095u), Dv = int((imt >> 12) & 255u);
    const int rloc = 2 * int((imt >> 20) & 63u);
    // gather levels k and k+1 (repeat loads hit the cache)
    double zlo[NV], ulo[NV], vlo[NV], dz[NV], du[NV], dv[NV], xr[NV], yr[NV], sv[NV];
    const double s0 = m.sigma[k], s1 = m.sigma[k + 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double4 g = m.geo[vidk[i]];
      if constexpr (TET) {   // corner positions relative to the first, and s
        const double4 g0 = m.geo[vidk[0]];
        xr[i] = g.x - g0.x;
        yr[i] = g.y - g0.y;
        sv[i] = m.sb[vidk[i]].x;
      }
      zlo[i] = g.z + s0 * g.w;
      dz[i] = (g.z + s1 * g.w) - zlo[i];
      const double2 a0 = *reinterpret_cast<const double2 *>(U + 2 * (int64_t(vidk[i]) * (L + 1) + k));
      const double2 a1 = *reinterpret_cast<const double2 *>(U + 2 * (int64_t(vidk[i]) * (L + 1) + k + 1));
      ulo[i] = a0.x; vlo[i] = a0.y;
      du[i] = a1.x - a0.x;
      dv[i] = a1.y - a0.y;
    }
    // wedges: x/y slopes of z, u, v at fixed zeta are (level-k sum) + zeta (increment sum)
    double HS[12];
    if constexpr (NV == 3 && !TET) {
#pragma unroll
      for (int h = 0; h < 12; ++h) HS[h] = 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        HS[0] = fma(lxc[i], zlo[i], HS[0]); HS[1] = fma(lxc[i], dz[i], HS[1]);
        HS[2] = fma(lyc[i], zlo[i], HS[2]); HS[3] = fma(lyc[i], dz[i], HS[3]);
        HS[4] = fma(lxc[i], ulo[i], HS[4]); HS[5] = fma(lxc[i], du[i], HS[5]);
        HS[6] = fma(lyc[i], ulo[i], HS[6]); HS[7] = fma(lyc[i], du[i], HS[7]);
        HS[8] = fma(lxc[i], vlo[i], HS[8]); HS[9] = fma(lxc[i], dv[i], HS[9]);
        HS[10] = fma(lyc[i], vlo[i], HS[10]); HS[11] = fma(lyc[i], dv[i], HS[11]);
      }
    }

    // residual rows of v's lower (index 0) and upper (index 1) node, and their tangents:
    // Jx[a][c][d][j][lev] = d R_(a,c) / d U_(node (j, lev), d)
    double Rb0 = 0, Rb1 = 0, Rt0 = 0, Rt1 = 0;
    AT Jx[2][2][2][NV][2];
    if constexpr (JAC) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int j = 0; j < NV; ++j) { Jx[a][c][d][j][0] = AT(0); Jx[a][c][d][j][1] = AT(0); }
    }

    AT FA[2][4][2], FH[2][4][2], FB[2][4][3];
    if constexpr (TET) {
      tet_layer<AT, JAC, N3>(m, al, picard, xr, yr, zlo, dz, ulo, du, vlo, dv, sv, Rb0, Rb1, Rt0, Rt1, Jx);
    } else if constexpr (NV == 3) {
      // Wedges.  The residual-only kernel runs the same loop without the tangents, so
      // both kernels produce the same residual bits.  The tangents are accumulated in
      // factorised form.  Every tangent
      // entry is sum_q L_q . b_q, where L_q (3 numbers per row node a and component pair
      // cd) depends on the row only and b_q is the column node's gradient.  For a wedge
      // column j, b = l0 h_j - lam_j p at the lower level and l1 h_j + lam_j p at the
      // upper one, with h_j = (dN_j/dx, dN_j/dy, 0) constant over the cell and
      // p = (d zeta/dx, d zeta/dy, d zeta/dz) the same for all j.  So it suffices to sum
      // l0 L and L (x, y parts) over all points, and L . p per triangle point; the six
      // column blocks are formed after the loop.
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int cd = 0; cd < 4; ++cd) {
          FA[a][cd][0] = FA[a][cd][1] = AT(0);
          FH[a][cd][0] = FH[a][cd][1] = AT(0);
          FB[a][cd][0] = FB[a][cd][1] = FB[a][cd][2] = AT(0);
        }
#pragma unroll
      for (int tp = 0; tp < 3; ++tp) {
        // the two points above triangle point tp share lam, z_zeta and the u, v increments
        double zze = 0, dum = 0, dvm = 0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          const double li = Q.lam[tp][i];
          zze = fma(li, dz[i], zze);
          dum = fma(li, du[i], dum);
          dvm = fma(li, dv[i], dvm);
        }
        const double iz = rcp64(zze);
        const double lam_a = ROT ? Q.lam[tp][0] : sel4(al, Q.lam[tp][0], Q.lam[tp][1], Q.lam[tp][2], 0.0);
        const double uz = iz * dum, vz = iz * dvm;
#pragma unroll 1
        for (int zi = 0; zi < 2; ++zi) {
          const int q = tp + 3 * zi;
          const double zeta = Q.zeta[q], l0 = 1.0 - zeta, l1 = zeta;
          const double zxs = fma(zeta, HS[1], HS[0]), zys = fma(zeta, HS[3], HS[2]);
          const double ucx = fma(zeta, HS[5], HS[4]), ucy = fma(zeta, HS[7], HS[6]);
          const double vcx = fma(zeta, HS[9], HS[8]), vcy = fma(zeta, HS[11], HS[10]);
          const double px = -zxs * iz, py = -zys * iz;        // d zeta / dx, d zeta / dy
          const double W = Q.w[q] * detc * zze;
          const double ux = ucx + px * dum, uy = ucy + py * dum;
          const double vx = vcx + px * dvm, vy = vcy + py * dvm;
          const double exx = ux, eyy = vy, exy = 0.5 * (uy + vx), exz = 0.5 * uz, eyz = 0.5 * vz;
          const double qq = exx * exx + eyy * eyy + exx * eyy + exy * exy + exz * exz + eyz * eyz;
          const double qe = qq + m.eps0_sq;
          double mu;
          if constexpr (N3) mu = m.visc_pref * rcbrt64(qe);
          else mu = m.visc_pref * powq(qe, m.visc_exp);
          const double s2 = 2.0 * mu * W;
          const double t2 = picard ? 0.0 : 2.0 * (m.visc_exp * mu * rcp64(qe)) * W;
          const double e1x = 2.0 * exx + eyy, e1y = exy, e1z = exz;
          const double e2x = exy, e2y = exx + 2.0 * eyy, e2z = eyz;
          const double gvx = W * m.rho_g * sxc, gvy = W * m.rho_g * syc;
          const double abx = l0 * lx_al - lam_a * px, aby = l0 * ly_al - lam_a * py, abz = -lam_a * iz;
          const double atx = l1 * lx_al + lam_a * px, aty = l1 * ly_al + lam_a * py, atz = lam_a * iz;
          const double gb0 = e1x * abx + e1y * aby + e1z * abz, gb1 = e2x * abx + e2y * aby + e2z * abz;
          const double gt0 = e1x * atx + e1y * aty + e1z * atz, gt1 = e2x * atx + e2y * aty + e2z * atz;
          const double nb = lam_a * l0, nt = lam_a * l1;
          Rb0 = fma(s2, gb0, fma(gvx, nb, Rb0));
          Rb1 = fma(s2, gb1, fma(gvy, nb, Rb1));
          Rt0 = fma(s2, gt0, fma(gvx, nt, Rt0));
          Rt1 = fma(s2, gt1, fma(gvy, nt, Rt1));
          if constexpr (!JAC) continue;
          const AT l0a = AT(l0), pxa = AT(px), pya = AT(py), iza = AT(iz);
          const AT e1xa = AT(e1x), e1ya = AT(e1y), e1za = AT(e1z);
          const AT e2xa = AT(e2x), e2ya = AT(e2y), e2za = AT(e2z);
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const AT Ax = AT(s2 * (a ? atx : abx)), Ay = AT(s2 * (a ? aty : aby)), Az = AT(s2 * (a ? atz : abz));
            const AT T0 = AT(t2 * (a ? gt0 : gb0)), T1 = AT(t2 * (a ? gt1 : gb1));
            const AT hAx = AT(0.5) * Ax, hAy = AT(0.5) * Ay, hAz = AT(0.5) * Az;
            // L for uu, uv, vu, vv: coefficients of (bx, by, bz) in d R_(a,c) / d U_(b,d)
            const AT Lx[4] = {fma(T0, e1xa, Ax + Ax), fma(T0, e2xa, hAy), fma(T1, e1xa, Ay), fma(T1, e2xa, hAx)};
            const AT Ly[4] = {fma(T0, e1ya, hAy), fma(T0, e2ya, Ax), fma(T1, e1ya, hAx), fma(T1, e2ya, Ay + Ay)};
            const AT Lz[4] = {fma(T0, e1za, hAz), T0 * e2za, T1 * e1za, fma(T1, e2za, hAz)};
#pragma unroll
            for (int cd = 0; cd < 4; ++cd) {
              FA[a][cd][0] = fma(l0a, Lx[cd], FA[a][cd][0]);
              FA[a][cd][1] = fma(l0a, Ly[cd], FA[a][cd][1]);
              FH[a][cd][0] += Lx[cd];
              FH[a][cd][1] += Ly[cd];
              FB[a][cd][tp] = fma(Lx[cd], pxa, fma(Ly[cd], pya, fma(Lz[cd], iza, FB[a][cd][tp])));
            }
          }
        }
      }
    } else {
#pragma unroll 1
      for (int q = 0; q < NQ; ++q) {
        const double zeta = Q.zeta[q], l0 = 1.0 - zeta, l1 = zeta;
        double lam[NV], lx[NV], ly[NV];
        double det, sx, sy;
#pragma unroll
        for (int i = 0; i < NV; ++i) lam[i] = Q.lam[q][i];
        if constexpr (NV == 3) {
#pragma unroll
          for (int i = 0; i < NV; ++i) { lx[i] = lxc[i]; ly[i] = lyc[i]; }
          det = detc; sx = sxc; sy = syc;
        } else {
          double x_xi = 0, x_eta = 0, y_xi = 0, y_eta = 0;
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            x_xi += xl[i] * Q.dlx[q][i]; x_eta += xl[i] * Q.dly[q][i];
            y_xi += yl[i] * Q.dlx[q][i]; y_eta += yl[i] * Q.dly[q][i];
          }
          det = x_xi * y_eta - x_eta * y_xi;
          const double iG = rcp64(det);
          const double i00 = y_eta * iG, i01 = -x_eta * iG, i10 = -y_xi * iG, i11 = x_xi * iG;
          sx = 0; sy = 0;
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            lx[i] = Q.dlx[q][i] * i00 + Q.dly[q][i] * i10;
            ly[i] = Q.dlx[q][i] * i01 + Q.dly[q][i] * i11;
            sx += su[i] * lx[i];
            sy += su[i] * ly[i];
          }
        }
        // vertical map: z_zeta and the slopes of z along x, y at fixed zeta
        double zze = 0, zxs, zys, ucx, ucy, vcx, vcy, dum = 0, dvm = 0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          zze = fma(lam[i], dz[i], zze);
          dum = fma(lam[i], du[i], dum);
          dvm = fma(lam[i], dv[i], dvm);
        }
        if constexpr (NV == 3) {
          zxs = fma(zeta, HS[1], HS[0]); zys = fma(zeta, HS[3], HS[2]);
          ucx = fma(zeta, HS[5], HS[4]); ucy = fma(zeta, HS[7], HS[6]);
          vcx = fma(zeta, HS[9], HS[8]); vcy = fma(zeta, HS[11], HS[10]);
        } else {
          zxs = zys = ucx = ucy = vcx = vcy = 0;
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            const double zc = fma(zeta, dz[i], zlo[i]);
            const double uc = fma(zeta, du[i], ulo[i]);
            const double vc = fma(zeta, dv[i], vlo[i]);
            zxs = fma(lx[i], zc, zxs); zys = fma(ly[i], zc, zys);
            ucx = fma(lx[i], uc, ucx); ucy = fma(ly[i], uc, ucy);
            vcx = fma(lx[i], vc, vcx); vcy = fma(ly[i], vc, vcy);
          }
        }
        const double iz = rcp64(zze);
        const double px = -zxs * iz, py = -zys * iz;        // d zeta / dx, d zeta / dy
        const double W = Q.w[q] * det * zze;
        // velocity gradient, strain rates, viscosity
        const double ux = ucx + px * dum, uy = ucy + py * dum, uz = iz * dum;
        const double vx = vcx + px * dvm, vy = vcy + py * dvm, vz = iz * dvm;
        const double exx = ux, eyy = vy, exy = 0.5 * (uy + vx), exz = 0.5 * uz, eyz = 0.5 * vz;
        const double qq = exx * exx + eyy * eyy + exx * eyy + exy * exy + exz * exz + eyz * eyz;
        const double qe = qq + m.eps0_sq;
        double mu;
        if constexpr (N3) mu = m.visc_pref * rcbrt64(qe);
        else mu = m.visc_pref * powq(qe, m.visc_exp);
        const double s2 = 2.0 * mu * W;
        const double t2 = picard ? 0.0 : 2.0 * (m.visc_exp * mu * rcp64(qe)) * W;
        const double e1x = 2.0 * exx + eyy, e1y = exy, e1z = exz;
        const double e2x = exy, e2y = exx + 2.0 * eyy, e2z = eyz;
        const double gvx = W * m.rho_g * sx, gvy = W * m.rho_g * sy;
        // v's own nodes in this cell: corner al at the lower and upper level
        const double lam_a = sel4(al, lam[0], lam[1], lam[2], lam[NV - 1]);
        double lxa, lya;
        if constexpr (NV == 3) { lxa = lx_al; lya = ly_al; }
        else { lxa = sel4(al, lx[0], lx[1], lx[2], lx[NV - 1]); lya = sel4(al, ly[0], ly[1], ly[2], ly[NV - 1]); }
        const double abx = l0 * lxa - lam_a * px, aby = l0 * lya - lam_a * py, abz = -lam_a * iz;
        const double atx = l1 * lxa + lam_a * px, aty = l1 * lya + lam_a * py, atz = lam_a * iz;
        const double gb0 = e1x * abx + e1y * aby + e1z * abz, gb1 = e2x * abx + e2y * aby + e2z * abz;
        const double gt0 = e1x * atx + e1y * aty + e1z * atz, gt1 = e2x * atx + e2y * aty + e2z * atz;
        const double nb = lam_a * l0, nt = lam_a * l1;     // v's basis functions at q
        Rb0 = fma(s2, gb0, fma(gvx, nb, Rb0));
        Rb1 = fma(s2, gb1, fma(gvy, nb, Rb1));
        Rt0 = fma(s2, gt0, fma(gvx, nt, Rt0));
        Rt1 = fma(s2, gt1, fma(gvy, nt, Rt1));
        if constexpr (JAC) {
          // row side: 2 mu W times the row node's gradient (with the constant factors of
          // d(eps_c . grad N_a)/dU folded into 2x copies here and 1/2 copies on the column
          // side; all scalings are exact), and 2 mu' W times its strain projection
          AT RA[2][7];
          {
            const AT s2a = AT(s2), t2a = AT(t2);
            const AT ax[2] = {AT(abx), AT(atx)}, ay[2] = {AT(aby), AT(aty)}, az[2] = {AT(abz), AT(atz)};
            const AT g0[2] = {AT(gb0), AT(gt0)}, g1[2] = {AT(gb1), AT(gt1)};
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const AT Ax = s2a * ax[a], Ay = s2a * ay[a];
              RA[a][0] = Ax; RA[a][1] = Ay; RA[a][2] = s2a * az[a];
              RA[a][3] = Ax + Ax; RA[a][4] = Ay + Ay;
              RA[a][5] = t2a * g0[a]; RA[a][6] = t2a * g1[a];
            }
          }
          // column side in the derivative type: d(grad N_b) and d(eps_e^2) along (b, u|v)
          const AT pxa = AT(px), pya = AT(py), izh = AT(0.5 * iz);
          const AT e1xa = AT(e1x), e1ya = AT(e1y), e1z2 = AT(2.0 * e1z);
          const AT e2xa = AT(e2x), e2ya = AT(e2y), e2z2 = AT(2.0 * e2z);
#pragma unroll
          for (int j = 0; j < NV; ++j) {
            const AT lxj = AT(lx[j]), lyj = AT(ly[j]), lmj = AT(lam[j]);
#pragma unroll
            for (int lev = 0; lev < 2; ++lev) {
              const AT ll = AT(lev ? l1 : l0);
              const AT dl = lev ? lmj : -lmj;
              const AT bx = fma(ll, lxj, dl * pxa), by = fma(ll, lyj, dl * pya), bzh = dl * izh;
              const AT bxh = AT(0.5) * bx, byh = AT(0.5) * by;
              const AT gu = fma(e1xa, bx, fma(e1ya, by, e1z2 * bzh));   // d(eps_e^2)/dU_(b,u)
              const AT gv = fma(e2xa, bx, fma(e2ya, by, e2z2 * bzh));   // d(eps_e^2)/dU_(b,v)
#pragma unroll
              for (int a = 0; a < 2; ++a) {
                AT &uu = Jx[a][0][0][j][lev], &uv = Jx[a][0][1][j][lev];
                AT &vu = Jx[a][1][0][j][lev], &vv = Jx[a][1][1][j][lev];
                const AT Ax = RA[a][0], Ay = RA[a][1], Az = RA[a][2], Ax2 = RA[a][3], Ay2 = RA[a][4];
                const AT T0 = RA[a][5], T1 = RA[a][6];
                uu = fma(Ax2, bx, uu); uu = fma(Ay, byh, uu); uu = fma(Az, bzh, uu); uu = fma(T0, gu, uu);
                uv = fma(Ax, by, uv); uv = fma(Ay, bxh, uv); uv = fma(T0, gv, uv);
                vu = fma(Ay, bx, vu); vu = fma(Ax, byh, vu); vu = fma(T1, gu, vu);
                vv = fma(Ax, bxh, vv); vv = fma(Ay2, by, vv); vv = fma(Az, bzh, vv); vv = fma(T1, gv, vv);
              }
            }
          }
        }
      }
  
    }

    // The window adds run at wave priority 1 and the copy-out at 2 (below): the other wave's
    // quadrature work then fills the LDS queue's gaps (about -1% each; priority for the adds
    // above the copy-out's, or for the quadrature loop, was slower).
    __builtin_amdgcn_s_setprio(1);
    // ---- add v's rows into the level windows ------------------------------------------------
    // (tetrahedra: every lane adds, lanes without an item add zeros to in-range entries; the
    // register allocator placed spills of live values inside the branch on `act` there)
    if (act || TET) {
      double *Rcur = Rw + cur * 2 * max_tv, *Rnxt = Rw + nxt * 2 * max_tv;
      lds_add(Rcur + rloc, Rb0);
      lds_add(Rcur + rloc + 1, Rb1);
      lds_add(Rnxt + rloc, Rt0);
      lds_add(Rnxt + rloc + 1, Rt1);
      if constexpr (JAC) {
        int rk[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) rk[i] = int((ipy >> (8 * i)) & 255u);
        const int nlk = nlev(k, L), nl1 = nlev(k + 1, L);
        const int offk = k > 0 ? 1 : 0;     // level k sits at window position 1 unless k = 0
        double *Wk = Jw + cur * max_slot + soff, *Wk1 = Jw + nxt * max_slot + soff;
        // each (row node, component pair)'s column blocks are added as soon as they are formed
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int cd = 0; cd < 4; ++cd) {
            const int c = cd >> 1, d = cd & 1;
            if constexpr (NV == 3 && !TET) {
              const AT Ux = FH[a][cd][0] - FA[a][cd][0], Uy = FH[a][cd][1] - FA[a][cd][1];
#pragma unroll
              for (int j = 0; j < NV; ++j) {
                const AT lam = fma(AT(Q.lam[0][j]), FB[a][cd][0],
                                   fma(AT(Q.lam[1][j]), FB[a][cd][1], AT(Q.lam[2][j]) * FB[a][cd][2]));
                const AT hx = AT(lxc[j]), hy = AT(lyc[j]);
                Jx[a][c][d][j][0] = fma(hx, FA[a][cd][0], fma(hy, FA[a][cd][1], -lam));
                Jx[a][c][d][j][1] = fma(hx, Ux, fma(hy, Uy, lam));
              }
            }
#pragma unroll
            for (int j = 0; j < NV; ++j)
#pragma unroll
              for (int lev = 0; lev < 2; ++lev) {
                if (a == 0) {
                  AT lo = Jx[0][c][d][j][lev];
                  if (CARRY && lev == 0) lo += carry[c][d][j];
                  if (CARRY0 && lev == 0 && j == 0 && k > 0) lo += carry0[2 * c + d];
                  lds_add(Wk + c * 2 * nlk * Dv + rk[j] * 2 * nlk + 2 * (lev + offk) + d, double(lo));
                } else if (CARRY && lev == 1 && k + 1 < L) {
                  carry[c][d][j] = Jx[1][c][d][j][1];
                } else if (CARRY0 && lev == 1 && j == 0 && k + 1 < L) {
                  carry0[2 * c + d] = double(Jx[1][c][d][0][1]);
                } else {
                  lds_add(Wk1 + c * 2 * nl1 * Dv + rk[j] * 2 * nl1 + 2 * lev + d, double(Jx[1][c][d][j][lev]));
                }
              }
          }
      }
    }
    wave_sync();

    // ---- level k is complete: copy it to its CSR rows and clear it for level k+2 ------------
    // Copy out four vertex columns at a time: all LDS reads of a batch are issued before
    // the first global store, so one LDS latency is exposed per batch, not per chunk.
    auto flush = [&](int lev_k, int slot) {
      const int nl = nlev(lev_k, L);
      const int lk = cumlev(lev_k);
      double *wb = Jw + slot * max_slot;   // 16-byte aligned, as is every column's slot
      for (int i0 = 0; i0 < nvt; i0 += 4) {
        if constexpr (JAC) {
          // each lane moves two consecutive entries: one 16-byte LDS read and one 16-byte
          // clearing write per column cover up to 128 entries (degree <= 10 at nl = 3)
          double2 val[4];
          int nn[4], so[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int ii = i0 + i < nvt ? i0 + i : nvt - 1;
            so[i] = __builtin_amdgcn_readlane(my_soff, ii);
            nn[i] = i0 + i < nvt ? 4 * nl * __builtin_amdgcn_readlane(my_deg, ii) : 0;
            const int e = 2 * lane;
            val[i] = *reinterpret_cast<const double2 *>(wb + so[i] + (e < nn[i] ? e : 0));
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (i0 + i >= nvt) break;
            const int ii = i0 + i;
            const int D = __builtin_amdgcn_readlane(my_deg, ii);
            const int64_t col = int64_t(unsigned(__builtin_amdgcn_readlane(my_col_lo, ii))) |
                                (int64_t(__builtin_amdgcn_readlane(my_col_hi, ii)) << 32);
            JT *dst = J + col + int64_t(4) * D * lk;
            double *src = wb + so[i];
            const int e = 2 * lane;   // nn is a multiple of 4, so e < nn implies e + 1 < nn
            if (e < nn[i]) {
              store2_nt(dst + e, val[i].x, val[i].y);
              *reinterpret_cast<double2 *>(src + e) = make_double2(0.0, 0.0);
            }
            for (int f = e + 2 * WAVE; f < nn[i]; f += 2 * WAVE) {
              const double2 w = *reinterpret_cast<const double2 *>(src + f);
              store2_nt(dst + f, w.x, w.y);
              *reinterpret_cast<double2 *>(src + f) = make_double2(0.0, 0.0);
            }
          }
        }
        if (lane < 8 && i0 + (lane >> 1) < nvt) {
          const int u = vb + i0 + (lane >> 1);
          double *rs = Rw + slot * 2 * max_tv + 2 * (u - vb) + (lane & 1);
          if (R) R[2 * (int64_t(u) * (L + 1) + lev_k) + (lane & 1)] = *rs;
          *rs = 0.0;
        }
      }
    };
    // The copy-out runs at raised wave priority: its LDS reads and streaming stores then issue
    // ahead of the other wave's quadrature work instead of queuing behind it (FP64 R+J -2%,
    // FP32 -2.5%; raising the gather instead was slower).
    __builtin_amdgcn_s_setprio(2);
    flush(k, cur);
    if (k == L - 1) flush(L, nxt);
    wave_sync();
    __builtin_amdgcn_s_setprio(0);

  }
}

template <int NV, bool JAC, class JT, bool N3, bool TET>
__global__ __launch_bounds__(WAVE, NV == 3 ? 2 : 1) void owner_kernel(MeshView m, const int4 *__restrict__ tasks,
                                                     const double *__restrict__ U, double *__restrict__ R,
                                                     JT *__restrict__ J, int picard, int max_slot,
                                                     int max_tv) {
  extern __shared__ __align__(16) unsigned char smem[];
  owner_task<NV, JAC, JT, N3, TET>(m, tasks[blockIdx.x], U, R, J, picard, max_slot, max_tv, smem);
}

// Persistent ensemble launch: each workgroup repeatedly takes the next (member, task) pair
// from a device counter until the combined task table is exhausted (every wave exits).
template <int NV, bool JAC, class JT, bool N3, bool TET>
__global__ __launch_bounds__(WAVE, NV == 3 ? 2 : 1) void ensemble_kernel(const EnsembleMember *__restrict__ mem,
                                                        const int4 *__restrict__ tasks, int n_tasks,
                                                        int *__restrict__ counter, int picard) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int ti = next;
    __syncthreads();
    if (ti >= n_tasks) break;
    const int4 task = tasks[ti];
    const EnsembleMember &e = mem[task.x];
    owner_task<NV, JAC, JT, N3, TET>(e.view, task, e.U, e.R, static_cast<JT *>(e.J), picard, e.max_slot,
                                     e.max_tv, smem);
  }
}

__global__ void fill_zero_kernel(uint4 *__restrict__ p, int64_t n16) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void fill_zero_tail_kernel(uint32_t *__restrict__ p, int64_t n4) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n4) p[i] = 0u;
}

// Ocean-front loads (memoised at upload) added to the residual rows of the front columns:
// one thread per (front vertex, level, component).
__global__ void front_add_kernel(int n_front, int L, const int32_t *__restrict__ vtx,
                                 const double *__restrict__ load, double *__restrict__ R) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = 2 * int64_t(L + 1);
  if (i >= n_front * per) return;
  const int64_t f = i / per, r = i - f * per;
  R[2 * int64_t(vtx[f]) * (L + 1) + r] += load[i];
}

bool g_tables_ready[64] = {};

fo_status ensure_tables(int device) {
  if (device >= 0 && device < 64 && g_tables_ready[device]) return FO_OK;
  static constexpr QTable tabs[2] = {make_table(3), make_table(4)};
  FO_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(kQ), tabs, sizeof(tabs)));
  if (device >= 0 && device < 64) g_tables_ready[device] = true;
  return FO_OK;
}

// LDS of one task: two level windows (Jacobian) and two residual windows
// Dynamic LDS of one task: the two Jacobian level windows, the two residual windows and,
// with a Jacobian, the per-lane carry slots (WAVE x 4 FP64) that follow them.
size_t window_bytes(bool jac, int max_slot, int max_tv) {
  return (jac ? 2 * size_t(max_slot) * sizeof(double) + size_t(WAVE) * 4 * sizeof(double) : 0) +
         2 * 2 * size_t(max_tv) * sizeof(double);
}

template <int NV, bool JAC, class JT, bool N3, bool TET>
fo_status launch_t(const fo_mesh *mesh, const double *U, double *R, JT *J, int kind, hipStream_t s) {
  const MeshView &m = mesh->view;
  const size_t lds = window_bytes(JAC, mesh->max_slot, mesh->max_task_verts);
  fo_status st = profile_begin(mesh, s);
  if (st != FO_OK) return st;
  hipLaunchKernelGGL((owner_kernel<NV, JAC, JT, N3, TET>), dim3(unsigned(mesh->n_tasks)), dim3(WAVE), lds, s, m,
                     mesh->tasks, U, R, J, kind == FO_JAC_PICARD ? 1 : 0, mesh->max_slot,
                     mesh->max_task_verts);
  FO_LAUNCH_CHECK("owner_kernel");
  return profile_end(mesh, s);
}

template <int NV, bool JAC, class JT, bool TET = false>
fo_status launch_n(const fo_mesh *mesh, const double *U, double *R, JT *J, int kind, hipStream_t s) {
  if (mesh->view.n_glen == 3.0) return launch_t<NV, JAC, JT, true, TET>(mesh, U, R, J, kind, s);
  return launch_t<NV, JAC, JT, false, TET>(mesh, U, R, J, kind, s);
}

template <int NV, bool JAC, class JT, bool N3, bool TET>
fo_status launch_ens_t(const EnsembleLaunch &E, int kind, hipStream_t s) {
  const size_t lds = window_bytes(JAC, E.max_slot, E.max_tv);
  auto kern = ensemble_kernel<NV, JAC, JT, N3, TET>;
  int per_cu = 0;
  FO_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVE, lds));
  if (per_cu < 1) per_cu = 1;
  int64_t grid = int64_t(E.n_cu) * per_cu;
  if (grid > E.n_tasks) grid = E.n_tasks;
  if (grid < 1) grid = 1;
  fo_status st = launch_fill_zero(E.counter, 16, s);
  if (st != FO_OK) return st;
  hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(WAVE), lds, s, E.members, E.tasks, E.n_tasks, E.counter,
                     kind == FO_JAC_PICARD ? 1 : 0);
  FO_LAUNCH_CHECK("ensemble_kernel");
  return FO_OK;
}

template <int NV, bool JAC, class JT, bool TET = false>
fo_status launch_ens_n(const EnsembleLaunch &E, int kind, hipStream_t s) {
  if (E.all_n3) return launch_ens_t<NV, JAC, JT, true, TET>(E, kind, s);
  return launch_ens_t<NV, JAC, JT, false, TET>(E, kind, s);
}

}  // namespace

fo_status launch_front_add(const MeshView &m, int32_t n_front, const int32_t *vtx, const double *load, double *R,
                           hipStream_t s) {
  if (n_front == 0 || R == nullptr) return FO_OK;
  const int64_t n = int64_t(n_front) * 2 * (m.L + 1);
  hipLaunchKernelGGL(front_add_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, int(n_front), int(m.L), vtx,
                     load, R);
  FO_LAUNCH_CHECK("front_add_kernel");
  return FO_OK;
}

fo_status launch_ensemble(const EnsembleLaunch &E, int dtype, int kind, bool want_jac, hipStream_t s) {
  fo_status st = ensure_tables(E.device);
  if (st != FO_OK) return st;
  if (E.tet) {
    if (!want_jac) return launch_ens_n<3, false, double, true>(E, kind, s);
    if (dtype == FO_F32) return launch_ens_n<3, true, float, true>(E, kind, s);
    return launch_ens_n<3, true, double, true>(E, kind, s);
  }
  if (!want_jac) {
    if (E.nv == 3) return launch_ens_n<3, false, double>(E, kind, s);
    return launch_ens_n<4, false, double>(E, kind, s);
  }
  if (dtype == FO_F32) {
    if (E.nv == 3) return launch_ens_n<3, true, float>(E, kind, s);
    return launch_ens_n<4, true, float>(E, kind, s);
  }
  if (E.nv == 3) return launch_ens_n<3, true, double>(E, kind, s);
  return launch_ens_n<4, true, double>(E, kind, s);
}

fo_status launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return FO_OK;
  if ((reinterpret_cast<uintptr_t>(p) & 15) != 0 || (bytes & 3) != 0)
    return fail(FO_EINVAL, "fill_zero: pointer must be 16-byte aligned and size a multiple of 4");
  const int64_t n16 = int64_t(bytes / 16);
  if (n16 > 0) {
    const int64_t want = (n16 + 255) / 256;
    const unsigned grid = unsigned(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint4 *>(p), n16);
    FO_LAUNCH_CHECK("fill_zero_kernel");
  }
  const int64_t rem4 = int64_t((bytes - size_t(n16) * 16) / 4);
  if (rem4 > 0) {
    hipLaunchKernelGGL(fill_zero_tail_kernel, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<uint32_t *>(static_cast<char *>(p) + n16 * 16), rem4);
    FO_LAUNCH_CHECK("fill_zero_tail_kernel");
  }
  return FO_OK;
}

fo_status launch_assemble(const fo_mesh *mesh, const double *U, double *R, void *J, int dtype,
                          int kind, bool want_jac, hipStream_t s) {
  fo_status st = launch_assemble_cells(mesh, U, R, J, dtype, kind, want_jac, s);
  if (st != FO_OK) return st;
  return launch_front_add(mesh->view, mesh->n_front, mesh->front_vtx, mesh->front_load, R, s);
}

fo_status launch_assemble_cells(const fo_mesh *mesh, const double *U, double *R, void *J, int dtype,
                                int kind, bool want_jac, hipStream_t s) {
  fo_status st = ensure_tables(mesh->device);
  if (st != FO_OK) return st;
  const int nv = mesh->view.nv;
  if (mesh->view.tet) {
    if (!want_jac) return launch_n<3, false, double, true>(mesh, U, R, nullptr, kind, s);
    if (dtype == FO_F32) return launch_n<3, true, float, true>(mesh, U, R, static_cast<float *>(J), kind, s);
    return launch_n<3, true, double, true>(mesh, U, R, static_cast<double *>(J), kind, s);
  }
  if (!want_jac) {
    if (nv == 3) return launch_n<3, false, double>(mesh, U, R, nullptr, kind, s);
    return launch_n<4, false, double>(mesh, U, R, nullptr, kind, s);
  }
  if (dtype == FO_F32) {
    if (nv == 3) return launch_n<3, true, float>(mesh, U, R, static_cast<float *>(J), kind, s);
    return launch_n<4, true, float>(mesh, U, R, static_cast<float *>(J), kind, s);
  }
  if (nv == 3) return launch_n<3, true, double>(mesh, U, R, static_cast<double *>(J), kind, s);
  return launch_n<4, true, double>(mesh, U, R, static_cast<double *>(J), kind, s);
}

}  // namespace fo
