// Cell-parallel assembly of the first-order Stokes residual and Jacobian on gfx950.
//
// Physics (arXiv:2204.04321 Sec. 2): momentum balance eq. (FOStokes) with the
// strain-rate vectors eps1 = (2 e_xx + e_yy, e_xy, e_xz), eps2 = (e_xy,
// e_xx + 2 e_yy, e_yz); Glen viscosity eq. (effvisc) with the effective strain
// rate eq. (effeps), regularised by eps0; stress-free surface; linear bed
// friction beta u.  Discrete residual eq. (residual), Jacobian eq. (linearsystem)
// by forward-mode AD (Sec. 3.2): one derivative direction per element dof.
//
// Work decomposition (one "team" of 16 lanes per cell, 4 cells per wave64):
//   gather   every lane of the team reads the cell's nodal data (same addresses);
//   primal   lane q < NQ evaluates quadrature point q: geometry, basis gradients,
//            strain rates, viscosity and its derivative; results go to LDS;
//   tangents lane j < NDOF is derivative lane j: it seeds dU = e_j and pushes the
//            tangent through strain rate -> eps_e^2 -> mu -> element residual,
//            producing column j of the element Jacobian (and residual entry j);
//   scatter  lane j adds its residual entry and Jacobian column into the CSR
//            values with hardware FP64/FP32 atomics.
// Slots in the CSR are computed arithmetically from the column-major numbering:
// row (vertex a, level kr, comp c) starts at colptr[a] + 4 D_a cumlev(kr)
// + c 2 nlev(kr) D_a; column (vertex b, level kc, comp d) sits at
// rank(a,b) 2 nlev(kr) + 2 (kc - max(kr-1, 0)) + d within it.
#include <hip/hip_runtime.h>

#include "fo_internal.h"

namespace fo {
namespace {

constexpr int TEAM = 16;
constexpr int BLOCK = 256;
constexpr int TEAMS_PER_BLOCK = BLOCK / TEAM;

constexpr double G1 = 0.21132486540518711775;   // 1/2 - 1/(2 sqrt 3)
constexpr double G2 = 0.78867513459481288225;   // 1/2 + 1/(2 sqrt 3)

template <int NV>
struct Elem;
template <>
struct Elem<3> {  // wedge: P1 triangle x linear in zeta
  static constexpr int NPE = 6, NDOF = 12, NQ = 6, NQB = 3;
};
template <>
struct Elem<4> {  // hexahedron: bilinear quad x linear in zeta
  static constexpr int NPE = 8, NDOF = 16, NQ = 8, NQB = 4;
};

// Reference quadrature point q (reference cell [0,1]^2 or unit triangle, zeta in [0,1]).
template <int NV>
__device__ __forceinline__ void qpoint(int q, double &xi, double &eta, double &zeta, double &w) {
  if constexpr (NV == 3) {
    const int t = q % 3;
    xi = (t == 1) ? 2.0 / 3.0 : 1.0 / 6.0;
    eta = (t == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
    zeta = (q < 3) ? G1 : G2;
    w = 1.0 / 12.0;
  } else {
    xi = (q & 1) ? G2 : G1;
    eta = (q & 2) ? G2 : G1;
    zeta = (q & 4) ? G2 : G1;
    w = 0.125;
  }
}

template <int NV>
__device__ __forceinline__ void bpoint(int r, double &xi, double &eta, double &w) {
  if constexpr (NV == 3) {
    xi = (r == 1) ? 2.0 / 3.0 : 1.0 / 6.0;
    eta = (r == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
    w = 1.0 / 6.0;
  } else {
    xi = (r & 1) ? G2 : G1;
    eta = (r & 2) ? G2 : G1;
    w = 0.25;
  }
}

// 2D basis values and reference derivatives.
template <int NV>
__device__ __forceinline__ void basis2d(double xi, double eta, double *lam, double *dx, double *dy) {
  if constexpr (NV == 3) {
    lam[0] = 1.0 - xi - eta; lam[1] = xi; lam[2] = eta;
    dx[0] = -1.0; dx[1] = 1.0; dx[2] = 0.0;
    dy[0] = -1.0; dy[1] = 0.0; dy[2] = 1.0;
  } else {
    const double mx = 1.0 - xi, my = 1.0 - eta;
    lam[0] = mx * my; lam[1] = xi * my; lam[2] = xi * eta; lam[3] = mx * eta;
    dx[0] = -my; dx[1] = my; dx[2] = eta; dx[3] = -eta;
    dy[0] = -mx; dy[1] = -xi; dy[2] = xi; dy[3] = mx;
  }
}

__device__ __forceinline__ int nlev(int k, int L) { return (k == 0 || k == L) ? 2 : 3; }
__device__ __forceinline__ int cumlev(int k) { return k == 0 ? 0 : 3 * k - 1; }

template <class T>
__device__ __forceinline__ void atomic_add(T *p, T v) {
  unsafeAtomicAdd(p, v);
}

// Per quadrature point record in LDS (doubles): grad N_a (3 NPE), g_(a,c) = eps_c . grad N_a
// (2 NPE), then 2 mu W, 2 mu' W, W rho g s_x, W rho g s_y.
template <int NV>
struct Rec {
  static constexpr int NPE = Elem<NV>::NPE;
  static constexpr int GN = 0, GV = 3 * NPE, S2 = 5 * NPE, T2 = S2 + 1, GX = S2 + 2, GY = S2 + 3;
  static constexpr int SIZE = 5 * NPE + 4;
  // reduced-precision copy for FP32 derivative lanes: grad N, g, 2 mu W, 2 mu' W
  static constexpr int FSIZE = 5 * NPE + 2;
};

template <int NV, bool JAC, class JT>
__global__ __launch_bounds__(BLOCK) void assemble_kernel(MeshView m, const double *__restrict__ U,
                                                         double *__restrict__ R, JT *__restrict__ J,
                                                         int picard) {
  using E = Elem<NV>;
  using RC = Rec<NV>;
  constexpr int NPE = E::NPE, NDOF = E::NDOF, NQ = E::NQ, NQB = E::NQB;
  constexpr bool F32 = JAC && sizeof(JT) == 4;
  __shared__ double lds[TEAMS_PER_BLOCK * NQ * RC::SIZE];
  __shared__ float ldsf[F32 ? TEAMS_PER_BLOCK * NQ * RC::FSIZE : 1];

  const int team = threadIdx.x / TEAM;
  const int lane = threadIdx.x % TEAM;
  const int64_t cell = int64_t(blockIdx.x) * TEAMS_PER_BLOCK + team;
  const bool active = cell < m.n_cells;
  const int L = m.L;
  const int64_t c = active ? cell : 0;
  const int t = int(c / L);
  const int k = int(c - int64_t(t) * L);

  // ---- gather (all lanes of the team, identical addresses) -----------------------------
  int vid[NV];
  double xl[NV], yl[NV], zb[NV], zt[NV], su[NV], bet[NV];
  double uu[NPE], vv[NPE];
  const double sk = m.sigma[k], sk1 = m.sigma[k + 1];
  double x0 = 0.0, y0 = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    vid[i] = m.cells[int64_t(t) * NV + i];
    const double4 gm = m.geo[vid[i]];
    const double2 sbv = m.sb[vid[i]];
    if (i == 0) { x0 = gm.x; y0 = gm.y; }
    xl[i] = gm.x - x0;              // local coordinates: differences of large numbers once
    yl[i] = gm.y - y0;
    zb[i] = gm.z + sk * gm.w;
    zt[i] = gm.z + sk1 * gm.w;
    su[i] = sbv.x;
    bet[i] = sbv.y;
    const int64_t nb = int64_t(vid[i]) * (L + 1) + k;
    const double2 ub = *reinterpret_cast<const double2 *>(U + 2 * nb);
    const double2 ut = *reinterpret_cast<const double2 *>(U + 2 * nb + 2);
    uu[i] = ub.x; vv[i] = ub.y;
    uu[NV + i] = ut.x; vv[NV + i] = ut.y;
  }

  double *rec = lds + team * NQ * RC::SIZE;
  float *recf = ldsf + (F32 ? team * NQ * RC::FSIZE : 0);

  // ---- primal: lane q evaluates quadrature point q ----------------------------------------
  if (lane < NQ) {
    double xi, eta, zeta, w;
    qpoint<NV>(lane, xi, eta, zeta, w);
    double lam[NV], dlx[NV], dly[NV];
    basis2d<NV>(xi, eta, lam, dlx, dly);
    const double l0 = 1.0 - zeta, l1 = zeta;
    double x_xi = 0, x_eta = 0, y_xi = 0, y_eta = 0, z_xi = 0, z_eta = 0, z_ze = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double zc = l0 * zb[i] + l1 * zt[i];
      x_xi += xl[i] * dlx[i]; x_eta += xl[i] * dly[i];
      y_xi += yl[i] * dlx[i]; y_eta += yl[i] * dly[i];
      z_xi += zc * dlx[i];    z_eta += zc * dly[i];
      z_ze += lam[i] * (zt[i] - zb[i]);
    }
    const double detG = x_xi * y_eta - x_eta * y_xi;
    const double iG = 1.0 / detG;
    const double i00 = y_eta * iG, i01 = -x_eta * iG, i10 = -y_xi * iG, i11 = x_xi * iG;
    const double izz = 1.0 / z_ze;
    const double zx = -(z_xi * i00 + z_eta * i10) * izz;   // d zeta / dx
    const double zy = -(z_xi * i01 + z_eta * i11) * izz;   // d zeta / dy
    const double W = w * detG * z_ze;
    double gx[NPE], gy[NPE], gz[NPE];
    double ux = 0, uy = 0, uz = 0, vx = 0, vy = 0, vz = 0, sx = 0, sy = 0;
#pragma unroll
    for (int a = 0; a < NPE; ++a) {
      const int i = a % NV;
      const double ll = (a < NV) ? l0 : l1;
      const double dl = (a < NV) ? -1.0 : 1.0;
      const double nxi = dlx[i] * ll, neta = dly[i] * ll, nze = lam[i] * dl;
      gx[a] = nxi * i00 + neta * i10 + nze * zx;
      gy[a] = nxi * i01 + neta * i11 + nze * zy;
      gz[a] = nze * izz;
      ux += uu[a] * gx[a]; uy += uu[a] * gy[a]; uz += uu[a] * gz[a];
      vx += vv[a] * gx[a]; vy += vv[a] * gy[a]; vz += vv[a] * gz[a];
      sx += su[i] * gx[a]; sy += su[i] * gy[a];
    }
    const double exx = ux, eyy = vy, exy = 0.5 * (uy + vx), exz = 0.5 * uz, eyz = 0.5 * vz;
    const double q = exx * exx + eyy * eyy + exx * eyy + exy * exy + exz * exz + eyz * eyz;
    const double qe = q + m.eps0_sq;
    const double mu = m.visc_pref * pow(qe, m.visc_exp);
    const double dmu = m.visc_exp * mu / qe;
    const double e1x = 2.0 * exx + eyy, e1y = exy, e1z = exz;
    const double e2x = exy, e2y = exx + 2.0 * eyy, e2z = eyz;
    double *P = rec + lane * RC::SIZE;
#pragma unroll
    for (int a = 0; a < NPE; ++a) {
      P[RC::GN + 3 * a + 0] = gx[a];
      P[RC::GN + 3 * a + 1] = gy[a];
      P[RC::GN + 3 * a + 2] = gz[a];
      P[RC::GV + 2 * a + 0] = e1x * gx[a] + e1y * gy[a] + e1z * gz[a];
      P[RC::GV + 2 * a + 1] = e2x * gx[a] + e2y * gy[a] + e2z * gz[a];
    }
    P[RC::S2] = 2.0 * mu * W;
    P[RC::T2] = picard ? 0.0 : 2.0 * dmu * W;
    P[RC::GX] = W * m.rho_g * sx;
    P[RC::GY] = W * m.rho_g * sy;
    if constexpr (F32) {
      float *Pf = recf + lane * RC::FSIZE;
#pragma unroll
      for (int i = 0; i < 5 * NPE + 2; ++i) Pf[i] = float(P[i]);
    }
  }
  __syncthreads();

  // ---- tangents: lane j = element dof (b, d) ---------------------------------------------
  const int j = lane;
  const int b = j >> 1, d = j & 1;
  const bool jlane = active && j < NDOF;
  const int bj = jlane ? b : 0;
  using AT = typename std::conditional<F32, float, double>::type;
  double res = 0.0;
  AT col[NDOF];
#pragma unroll
  for (int i = 0; i < NDOF; ++i) col[i] = AT(0);

#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const double *P = rec + q * RC::SIZE;
    double xi, eta, zeta, w;
    qpoint<NV>(q, xi, eta, zeta, w);
    double lam[NV], dlx[NV], dly[NV];
    basis2d<NV>(xi, eta, lam, dlx, dly);
    const double Nb = lam[bj % NV] * ((bj < NV) ? (1.0 - zeta) : zeta);
    const double gbd = P[RC::GV + 2 * bj + d];
    res += P[RC::S2] * gbd + P[RC::GX + d] * Nb;
    if constexpr (JAC) {
      const AT *Q;
      if constexpr (F32) Q = recf + q * RC::FSIZE; else Q = P;
      const AT bx = Q[RC::GN + 3 * bj], by = Q[RC::GN + 3 * bj + 1], bz = Q[RC::GN + 3 * bj + 2];
      const AT s2 = Q[RC::S2];
      const AT tg = Q[RC::T2] * Q[RC::GV + 2 * bj + d];     // d(2 mu W) along e_j
      // tangent of eps1 / eps2 along e_j, scaled by 2 mu W
      const AT h = AT(0.5), two = AT(2);
      AT p1x, p1y, p1z, p2x, p2y, p2z;
      if (d == 0) { p1x = two * bx; p1y = h * by; p1z = h * bz; p2x = h * by; p2y = bx; p2z = AT(0); }
      else        { p1x = by; p1y = h * bx; p1z = AT(0); p2x = h * bx; p2y = two * by; p2z = h * bz; }
      p1x *= s2; p1y *= s2; p1z *= s2; p2x *= s2; p2y *= s2; p2z *= s2;
#pragma unroll
      for (int a = 0; a < NPE; ++a) {
        const AT ax = Q[RC::GN + 3 * a], ay = Q[RC::GN + 3 * a + 1], az = Q[RC::GN + 3 * a + 2];
        col[2 * a] += ax * p1x + ay * p1y + az * p1z + tg * Q[RC::GV + 2 * a];
        col[2 * a + 1] += ax * p2x + ay * p2y + az * p2z + tg * Q[RC::GV + 2 * a + 1];
      }
    }
  }

  // ---- bed friction on the lower face of bottom-layer cells -------------------------------
  if (k == 0) {
#pragma unroll
    for (int r = 0; r < NQB; ++r) {
      double xi, eta, w;
      bpoint<NV>(r, xi, eta, w);
      double lam[NV], dlx[NV], dly[NV];
      basis2d<NV>(xi, eta, lam, dlx, dly);
      double txx = 0, txy = 0, txz = 0, tyx = 0, tyy = 0, tyz = 0, br = 0, ur = 0;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        txx += xl[i] * dlx[i]; txy += yl[i] * dlx[i]; txz += zb[i] * dlx[i];
        tyx += xl[i] * dly[i]; tyy += yl[i] * dly[i]; tyz += zb[i] * dly[i];
        br += bet[i] * lam[i];
        ur += (d == 0 ? uu[i] : vv[i]) * lam[i];
      }
      const double nx = txy * tyz - txz * tyy, ny = txz * tyx - txx * tyz, nz = txx * tyy - txy * tyx;
      const double wb = w * sqrt(nx * nx + ny * ny + nz * nz) * br;
      if (bj < NV) {
        res += wb * ur * lam[bj];
        if constexpr (JAC) {
#pragma unroll
          for (int a = 0; a < NV; ++a) col[2 * a + d] += AT(wb * lam[a] * lam[bj]);
        }
      }
    }
  }

  if (!jlane) return;
  // ---- scatter -------------------------------------------------------------------------------
  const int lev_b = b / NV, beta_v = b % NV;
  const int kc = k + lev_b;
  const int64_t node_b = int64_t(vid[beta_v]) * (L + 1) + kc;
  if (R) atomic_add(R + 2 * node_b + d, res);
  if constexpr (JAC) {
    const uint8_t *rk = m.rank + int64_t(t) * NV * NV;
#pragma unroll
    for (int a = 0; a < NPE; ++a) {
      const int al = a % NV, kr = k + a / NV;
      const int va = vid[al];
      const int Da = m.deg[va];
      const int nl = nlev(kr, L);
      const int64_t rowblk = m.colptr[va] + int64_t(4) * Da * cumlev(kr);
      const int64_t off = int64_t(rk[al * NV + beta_v]) * 2 * nl + 2 * (kc - (kr > 0 ? kr - 1 : 0)) + d;
      atomic_add(J + rowblk + off, JT(col[2 * a]));
      atomic_add(J + rowblk + int64_t(2) * nl * Da + off, JT(col[2 * a + 1]));
    }
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

template <int NV, bool JAC, class JT>
fo_status launch_t(const fo_mesh *mesh, const double *U, double *R, JT *J, int kind, hipStream_t s) {
  const MeshView &m = mesh->view;
  const int64_t blocks = (m.n_cells + TEAMS_PER_BLOCK - 1) / TEAMS_PER_BLOCK;
  if (blocks > 0x7fffffff) return fail(FO_EINVAL, "assembly: too many cells for one launch");
  fo_status st = profile_begin(mesh, s);
  if (st != FO_OK) return st;
  hipLaunchKernelGGL((assemble_kernel<NV, JAC, JT>), dim3(unsigned(blocks)), dim3(BLOCK), 0, s, m, U,
                     R, J, kind == FO_JAC_PICARD ? 1 : 0);
  FO_LAUNCH_CHECK("assemble_kernel");
  return profile_end(mesh, s);
}

}  // namespace

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
  const MeshView &m = mesh->view;
  fo_status st;
  if (R && (st = launch_fill_zero(R, sizeof(double) * m.n_dofs, s)) != FO_OK) return st;
  if (!want_jac) {
    if (m.nv == 3) return launch_t<3, false, double>(mesh, U, R, nullptr, kind, s);
    return launch_t<4, false, double>(mesh, U, R, nullptr, kind, s);
  }
  const size_t esz = dtype == FO_F32 ? 4 : 8;
  if ((st = launch_fill_zero(J, esz * mesh->nnz, s)) != FO_OK) return st;
  if (dtype == FO_F32) {
    if (m.nv == 3) return launch_t<3, true, float>(mesh, U, R, static_cast<float *>(J), kind, s);
    return launch_t<4, true, float>(mesh, U, R, static_cast<float *>(J), kind, s);
  }
  if (m.nv == 3) return launch_t<3, true, double>(mesh, U, R, static_cast<double *>(J), kind, s);
  return launch_t<4, true, double>(mesh, U, R, static_cast<double *>(J), kind, s);
}

}  // namespace fo
