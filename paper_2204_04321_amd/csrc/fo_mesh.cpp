// Host side of mesh upload: validation, column-major numbering, neighbour lists,
// per-cell rank tables and the CSR layout of the Jacobian (memoised once per
// mesh, arXiv:2204.04321 Sec. 4.1), plus the small C ABI entry points that do
// not launch assembly kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fo_internal.h"

namespace fo {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

fo_status fail(fo_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

template <class T>
static fo_status dev_upload(T **dst, const T *src, size_t count, hipStream_t s) {
  *dst = nullptr;
  if (count == 0) return FO_OK;
  if (hipMalloc(reinterpret_cast<void **>(dst), count * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    return fail(FO_ENOMEM, "hipMalloc failed for a mesh table");
  }
  if (src) FO_HIP_TRY(hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
  return FO_OK;
}

static void release_events(fo_mesh *m) {
  for (auto &e : m->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  m->events.clear();
  m->n_recorded = 0;
}

fo_status profile_begin(const fo_mesh *cm, hipStream_t s) {
  fo_mesh *m = const_cast<fo_mesh *>(cm);
  if (!m->profiling) return FO_OK;
  if (m->n_recorded == m->events.size()) {
    std::pair<hipEvent_t, hipEvent_t> e;
    FO_HIP_TRY(hipEventCreate(&e.first));
    FO_HIP_TRY(hipEventCreate(&e.second));
    m->events.push_back(e);
  }
  FO_HIP_TRY(hipEventRecord(m->events[m->n_recorded].first, s));
  return FO_OK;
}

fo_status profile_end(const fo_mesh *cm, hipStream_t s) {
  fo_mesh *m = const_cast<fo_mesh *>(cm);
  if (!m->profiling) return FO_OK;
  FO_HIP_TRY(hipEventRecord(m->events[m->n_recorded].second, s));
  m->n_recorded++;
  return FO_OK;
}

static void free_mesh(fo_mesh *m) {
  if (!m) return;
  release_events(m);
  void *ptrs[] = {m->geo, m->sb, m->colptr, m->deg, m->cells, m->rank, m->sigma,
                  m->nbr_ptr, m->nbr_idx, m->self_rank, m->vc_ptr, m->vc_idx, m->vc_pos,
                  m->item_vtx, m->slot_off, m->item_rank, m->tasks, m->rowptr, m->colidx,
                  m->front_vtx, m->front_load};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

}  // namespace fo

using namespace fo;

extern "C" const char *fo_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *fo_status_string(fo_status s) {
  switch (s) {
    case FO_OK: return "ok";
    case FO_EINVAL: return "invalid argument";
    case FO_ENOMEM: return "out of memory";
    case FO_EDEVICE: return "device error";
    case FO_EDEGENERATE: return "degenerate mesh";
    case FO_ENONFINITE: return "non-finite value";
    case FO_ENOTCONV: return "not converged";
  }
  return "unknown status";
}

extern "C" fo_status fo_mesh_create(const fo_mesh_desc *d, void *stream, fo_mesh **out) {
  if (!out) return fail(FO_EINVAL, "fo_mesh_create: out is NULL");
  *out = nullptr;
  if (!d) return fail(FO_EINVAL, "fo_mesh_create: desc is NULL");
  if (d->elem != FO_WEDGE6 && d->elem != FO_HEX8 && d->elem != FO_TET4)
    return fail(FO_EINVAL, "fo_mesh_create: elem must be FO_WEDGE6, FO_TET4 or FO_HEX8");
  const int nv = d->elem == FO_HEX8 ? 4 : 3;
  const int64_t V = d->n_base_verts, T = d->n_base_cells, L = d->n_layers;
  if (V < nv || T < 1 || L < 1) return fail(FO_EINVAL, "fo_mesh_create: need V >= 3|4, T >= 1, L >= 1");
  if (!d->base_xy || !d->base_cells || !d->surface || !d->thickness || !d->beta)
    return fail(FO_EINVAL, "fo_mesh_create: a required host array is NULL");
  if (!(d->A > 0) || !(d->n >= 1) || !(d->rho > 0) || !(d->g > 0) || !(d->eps0 >= 0) ||
      !std::isfinite(d->A) || !std::isfinite(d->n) || !std::isfinite(d->rho) ||
      !std::isfinite(d->g) || !std::isfinite(d->eps0))
    return fail(FO_EINVAL, "fo_mesh_create: constants must be finite with A > 0, n >= 1, rho > 0, g > 0, eps0 >= 0");
  const int64_t n_dofs = 2 * V * (L + 1);
  if (n_dofs >= (int64_t(1) << 31)) return fail(FO_EINVAL, "fo_mesh_create: more than 2^31 dofs");

  std::vector<double> sig(L + 1);
  if (d->sigma) {
    for (int64_t k = 0; k <= L; ++k) sig[k] = d->sigma[k];
    if (sig[0] != 0.0 || sig[L] != 1.0)
      return fail(FO_EDEGENERATE, "fo_mesh_create: sigma must run from 0 to 1");
    for (int64_t k = 0; k < L; ++k)
      if (!(sig[k + 1] > sig[k])) return fail(FO_EDEGENERATE, "fo_mesh_create: sigma must increase");
  } else {
    for (int64_t k = 0; k <= L; ++k) sig[k] = double(k) / double(L);
  }
  for (int64_t v = 0; v < V; ++v) {
    const double x = d->base_xy[2 * v], y = d->base_xy[2 * v + 1];
    if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(d->surface[v]))
      return fail(FO_EDEGENERATE, "fo_mesh_create: non-finite coordinate or surface at vertex " + std::to_string(v));
    if (!(d->thickness[v] > 0) || !std::isfinite(d->thickness[v]))
      return fail(FO_EDEGENERATE, "fo_mesh_create: thickness must be > 0 at vertex " + std::to_string(v));
    if (!(d->beta[v] >= 0) || !std::isfinite(d->beta[v]))
      return fail(FO_EDEGENERATE, "fo_mesh_create: beta must be finite and >= 0 at vertex " + std::to_string(v));
  }
  const int32_t *C = d->base_cells;
  const double *xy = d->base_xy;
  std::vector<int32_t> front_vtx;
  std::vector<double> front_load;
  for (int64_t t = 0; t < T; ++t) {
    for (int a = 0; a < nv; ++a) {
      const int32_t va = C[t * nv + a];
      if (va < 0 || va >= V) return fail(FO_EINVAL, "fo_mesh_create: cell " + std::to_string(t) + " has a vertex out of range");
      for (int b = 0; b < a; ++b)
        if (C[t * nv + b] == va) return fail(FO_EDEGENERATE, "fo_mesh_create: repeated vertex in cell " + std::to_string(t));
    }
    // every corner turns left: positive area (triangles), strictly convex CCW (quads)
    for (int a = 0; a < nv; ++a) {
      const int32_t p = C[t * nv + (a + nv - 1) % nv], q = C[t * nv + a], r = C[t * nv + (a + 1) % nv];
      const double ux = xy[2 * q] - xy[2 * p], uy = xy[2 * q + 1] - xy[2 * p + 1];
      const double wx = xy[2 * r] - xy[2 * q], wy = xy[2 * r + 1] - xy[2 * q + 1];
      if (!(ux * wy - uy * wx > 0))
        return fail(FO_EDEGENERATE, "fo_mesh_create: cell " + std::to_string(t) + " is not counter-clockwise/convex");
    }
  }

  {
    fo_status fst = build_front_loads(d, sig, front_vtx, front_load);
    if (fst != FO_OK) return fst;
  }

  // vertex -> base cells (ordered by cell id): the owner-computes work items
  std::vector<int32_t> vc_ptr(V + 1, 0), vc_idx(size_t(T) * nv), item_vtx(size_t(T) * nv);
  std::vector<uint8_t> vc_pos(size_t(T) * nv);
  for (int64_t i = 0; i < T * nv; ++i) vc_ptr[C[i] + 1]++;
  for (int64_t v = 0; v < V; ++v) vc_ptr[v + 1] += vc_ptr[v];
  {
    std::vector<int32_t> fillp(vc_ptr.begin(), vc_ptr.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int a = 0; a < nv; ++a) {
        const int32_t v = C[t * nv + a];
        const int32_t p = fillp[v]++;
        vc_idx[p] = int32_t(t);
        vc_pos[p] = uint8_t(a);
        item_vtx[p] = v;
      }
  }
  // neighbour lists: vertices sharing a base cell (each vertex neighbours itself), built
  // column by column from the vertex's cells with a last-seen marker, then sorted (short
  // lists: insertion sort)
  std::vector<int32_t> nbr_ptr(V + 1, 0), nbr_idx;
  nbr_idx.reserve(size_t(V) * 8);
  {
    std::vector<int32_t> mark(V, -1);
    for (int64_t v = 0; v < V; ++v) {
      const size_t b0 = nbr_idx.size();
      nbr_idx.push_back(int32_t(v));
      mark[v] = int32_t(v);
      for (int32_t i = vc_ptr[v]; i < vc_ptr[v + 1]; ++i) {
        const int64_t t = vc_idx[i];
        for (int a = 0; a < nv; ++a) {
          const int32_t w = C[t * nv + a];
          if (mark[w] != int32_t(v)) {
            mark[w] = int32_t(v);
            nbr_idx.push_back(w);
          }
        }
      }
      for (size_t i = b0 + 1; i < nbr_idx.size(); ++i) {
        const int32_t x = nbr_idx[i];
        size_t j = i;
        for (; j > b0 && nbr_idx[j - 1] > x; --j) nbr_idx[j] = nbr_idx[j - 1];
        nbr_idx[j] = x;
      }
      nbr_ptr[v + 1] = int32_t(nbr_idx.size());
    }
  }
  std::vector<int32_t> deg(V), self_rank(V);
  std::vector<int64_t> colptr(V + 1, 0);
  for (int64_t v = 0; v < V; ++v) {
    deg[v] = nbr_ptr[v + 1] - nbr_ptr[v];
    self_rank[v] = int32_t(std::lower_bound(nbr_idx.data() + nbr_ptr[v], nbr_idx.data() + nbr_ptr[v + 1],
                                            int32_t(v)) - (nbr_idx.data() + nbr_ptr[v]));
    colptr[v + 1] = colptr[v] + 4 * int64_t(deg[v]) * (3 * L + 1);
  }
  std::vector<uint8_t> rank(size_t(T) * nv * nv);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < nv; ++a) {
      const int32_t va = C[t * nv + a];
      const int32_t *beg = nbr_idx.data() + nbr_ptr[va], *end = nbr_idx.data() + nbr_ptr[va + 1];
      for (int b = 0; b < nv; ++b) {
        const int32_t *it = std::lower_bound(beg, end, C[t * nv + b]);
        if (it - beg > 255) return fail(FO_EINVAL, "fo_mesh_create: vertex degree above 255");
        rank[(t * nv + a) * nv + b] = uint8_t(it - beg);
      }
    }
  // wave tasks: runs of consecutive vertex columns with at most 64 items (one lane each)
  // whose level windows (12 D entries per vertex) fit the per-wave LDS budget
  // kMaxSlot: two level windows of at most 1080 FP64 entries, the residual windows and the
  // per-lane carry slots (2 KB) keep a wave's LDS under 20 KB, so that eight waves share a
  // compute unit
  constexpr int kMaxItems = 64, kMaxSlot = 1080;
  std::vector<int4> tasks;
  std::vector<int32_t> slot_off(V);
  int32_t max_slot = 0, max_tv = 0;
  {
    int32_t vb = 0, items = 0, slot = 0;
    for (int32_t v = 0; v < int32_t(V); ++v) {
      const int32_t ni = vc_ptr[v + 1] - vc_ptr[v];
      const int32_t sz = 12 * deg[v];
      if (ni == 0)
        return fail(FO_EDEGENERATE, "fo_mesh_create: vertex " + std::to_string(v) + " lies in no base cell");
      if (ni > kMaxItems)
        return fail(FO_EINVAL, "fo_mesh_create: vertex " + std::to_string(v) + " lies in more than 64 base cells");
      if (sz > kMaxSlot)
        return fail(FO_EINVAL, "fo_mesh_create: vertex " + std::to_string(v) + " has more than 90 neighbouring vertices");
      if (v > vb && (items + ni > kMaxItems || slot + sz > kMaxSlot)) {
        tasks.push_back(make_int4(0, vb, v, vc_ptr[vb]));
        max_slot = std::max(max_slot, slot);
        max_tv = std::max(max_tv, v - vb);
        vb = v; items = 0; slot = 0;
      }
      slot_off[v] = slot;
      items += ni;
      slot += sz;
    }
    tasks.push_back(make_int4(0, vb, int32_t(V), vc_ptr[vb]));
    max_slot = std::max(max_slot, slot);
    max_tv = std::max(max_tv, int32_t(V) - vb);
  }
  // per item, the neighbour rank of each corner in the item vertex's list, 8 bits per corner
  std::vector<uint32_t> item_rank(size_t(T) * nv);
  for (int64_t p = 0; p < T * nv; ++p) {
    const int64_t t = vc_idx[p];
    const int a = vc_pos[p];
    uint32_t rx = 0;
    for (int b = 0; b < nv; ++b) rx |= uint32_t(rank[(t * nv + a) * nv + b]) << (8 * b);
    item_rank[p] = rx;
  }
  std::vector<double4> geo(V);
  std::vector<double2> sb(V);
  for (int64_t v = 0; v < V; ++v) {
    geo[v] = make_double4(xy[2 * v], xy[2 * v + 1], d->surface[v] - d->thickness[v], d->thickness[v]);
    sb[v] = make_double2(d->surface[v], d->beta[v]);
  }

  hipStream_t s = static_cast<hipStream_t>(stream);
  fo_mesh *m = new fo_mesh();
  (void)hipGetDevice(&m->device);
  m->elem = d->elem;
  m->nnz = colptr[V];
  fo_status st = FO_OK;
#define UP(dst, vec) if ((st = dev_upload(&m->dst, vec.data(), vec.size(), s)) != FO_OK) { free_mesh(m); return st; }
  UP(geo, geo);
  UP(sb, sb);
  UP(colptr, colptr);
  UP(deg, deg);
  UP(rank, rank);
  UP(sigma, sig);
  UP(nbr_ptr, nbr_ptr);
  UP(nbr_idx, nbr_idx);
  UP(self_rank, self_rank);
  UP(vc_ptr, vc_ptr);
  UP(vc_idx, vc_idx);
  UP(vc_pos, vc_pos);
  UP(item_vtx, item_vtx);
  UP(slot_off, slot_off);
  UP(item_rank, item_rank);
  UP(tasks, tasks);
  UP(front_vtx, front_vtx);
  UP(front_load, front_load);
  m->n_front = int32_t(front_vtx.size());
#undef UP
  if ((st = dev_upload(&m->cells, C, size_t(T) * nv, s)) != FO_OK) { free_mesh(m); return st; }
  if ((st = dev_upload<int64_t>(&m->rowptr, nullptr, size_t(n_dofs + 1), s)) != FO_OK) { free_mesh(m); return st; }
  if ((st = dev_upload<int32_t>(&m->colidx, nullptr, size_t(m->nnz), s)) != FO_OK) { free_mesh(m); return st; }

  MeshView &mv = m->view;
  mv.nv = nv;
  mv.tet = d->elem == FO_TET4 ? 1 : 0;
  mv.L = int32_t(L);
  mv.V = int32_t(V);
  mv.T = int32_t(T);
  mv.n_cells = T * L;
  mv.n_dofs = n_dofs;
  mv.geo = m->geo;
  mv.sb = m->sb;
  mv.colptr = m->colptr;
  mv.deg = m->deg;
  mv.cells = m->cells;
  mv.rank = m->rank;
  mv.sigma = m->sigma;
  mv.vc_ptr = m->vc_ptr;
  mv.vc_idx = m->vc_idx;
  mv.vc_pos = m->vc_pos;
  mv.item_vtx = m->item_vtx;
  mv.slot_off = m->slot_off;
  mv.item_rank = m->item_rank;
  m->n_tasks = int32_t(tasks.size());
  m->tasks_host = tasks;
  m->max_slot = max_slot;
  m->max_task_verts = max_tv;
  mv.rho_g = d->rho * d->g;
  mv.visc_pref = 0.5 * std::pow(d->A, -1.0 / d->n);
  mv.visc_exp = (1.0 - d->n) / (2.0 * d->n);
  mv.n_glen = d->n;
  mv.A = d->A;
  mv.eps0_sq = d->eps0 * d->eps0;

  if ((st = launch_pattern(m, s)) != FO_OK) { free_mesh(m); return st; }
  if (hipStreamSynchronize(s) != hipSuccess) {
    free_mesh(m);
    return fail(FO_EDEVICE, "fo_mesh_create: stream synchronisation failed");
  }
  *out = m;
  return FO_OK;
}

extern "C" void fo_mesh_destroy(fo_mesh *m) { free_mesh(m); }

extern "C" fo_status fo_profile_enable(fo_mesh *m, int32_t on) {
  if (!m) return fail(FO_EINVAL, "fo_profile_enable: mesh is NULL");
  if (!on) release_events(m);
  m->profiling = on != 0;
  m->n_recorded = 0;
  return FO_OK;
}

extern "C" fo_status fo_profile_read(fo_mesh *m, double *kernel_ms, int64_t *launches) {
  if (!m) return fail(FO_EINVAL, "fo_profile_read: mesh is NULL");
  double total = 0.0;
  for (size_t i = 0; i < m->n_recorded; ++i) {
    FO_HIP_TRY(hipEventSynchronize(m->events[i].second));
    float ms = 0.f;
    FO_HIP_TRY(hipEventElapsedTime(&ms, m->events[i].first, m->events[i].second));
    total += ms;
  }
  if (kernel_ms) *kernel_ms = total;
  if (launches) *launches = int64_t(m->n_recorded);
  m->n_recorded = 0;
  return FO_OK;
}

extern "C" fo_status fo_mesh_info(const fo_mesh *m, int64_t *n_nodes, int64_t *n_dofs,
                                  int64_t *n_cells, int64_t *nnz) {
  if (!m) return fail(FO_EINVAL, "fo_mesh_info: mesh is NULL");
  if (n_nodes) *n_nodes = m->view.n_dofs / 2;
  if (n_dofs) *n_dofs = m->view.n_dofs;
  if (n_cells) *n_cells = m->view.n_cells;
  if (nnz) *nnz = m->nnz;
  return FO_OK;
}

extern "C" fo_status fo_jacobian_pattern(const fo_mesh *m, int64_t *rowptr_dev, int32_t *colidx_dev,
                                         void *stream) {
  if (!m) return fail(FO_EINVAL, "fo_jacobian_pattern: mesh is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (rowptr_dev)
    FO_HIP_TRY(hipMemcpyAsync(rowptr_dev, m->rowptr, sizeof(int64_t) * (m->view.n_dofs + 1),
                              hipMemcpyDeviceToDevice, s));
  if (colidx_dev)
    FO_HIP_TRY(hipMemcpyAsync(colidx_dev, m->colidx, sizeof(int32_t) * m->nnz,
                              hipMemcpyDeviceToDevice, s));
  return FO_OK;
}

extern "C" fo_status fo_assemble_residual(const fo_mesh *m, const double *U, double *R, void *stream) {
  if (!m || !U || !R) return fail(FO_EINVAL, "fo_assemble_residual: NULL argument");
  if ((reinterpret_cast<uintptr_t>(U) & 15) || (reinterpret_cast<uintptr_t>(R) & 15))
    return fail(FO_EINVAL, "fo_assemble_residual: U and R must be 16-byte aligned");
  return launch_assemble(m, U, R, nullptr, FO_F64, FO_JAC_NEWTON, false, static_cast<hipStream_t>(stream));
}

extern "C" fo_status fo_assemble_jacobian(const fo_mesh *m, const double *U, double *R, void *J,
                                          int32_t dtype, int32_t kind, void *stream) {
  if (!m || !U || !J) return fail(FO_EINVAL, "fo_assemble_jacobian: NULL argument");
  if ((reinterpret_cast<uintptr_t>(U) & 15) || (reinterpret_cast<uintptr_t>(R) & 15) ||
      (reinterpret_cast<uintptr_t>(J) & 15))
    return fail(FO_EINVAL, "fo_assemble_jacobian: U, R and J must be 16-byte aligned");
  if (dtype != FO_F64 && dtype != FO_F32) return fail(FO_EINVAL, "fo_assemble_jacobian: bad dtype");
  if (kind != FO_JAC_NEWTON && kind != FO_JAC_PICARD) return fail(FO_EINVAL, "fo_assemble_jacobian: bad kind");
  return launch_assemble(m, U, R, J, dtype, kind, true, static_cast<hipStream_t>(stream));
}

extern "C" fo_status fo_initial_guess_sia(const fo_mesh *m, double *U, void *stream) {
  if (!m || !U) return fail(FO_EINVAL, "fo_initial_guess_sia: NULL argument");
  return launch_sia(m, U, static_cast<hipStream_t>(stream));
}
