// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fo_stokes.h"

namespace fo {

// Thread-local error message behind fo_last_error().
void set_error(const std::string &msg);
fo_status fail(fo_status s, const std::string &msg);

#define FO_HIP_TRY(expr)                                                               \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return ::fo::fail(FO_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
  } while (0)

#define FO_LAUNCH_CHECK(what)                                                          \
  do {                                                                                 \
    hipError_t _e = hipGetLastError();                                                 \
    if (_e != hipSuccess)                                                              \
      return ::fo::fail(FO_EDEVICE, std::string(what " launch failed: ") + hipGetErrorString(_e)); \
  } while (0)

// Device-side view of one extruded mesh (plain pointers; passed by value to kernels).
struct MeshView {
  int32_t nv;        // vertices per base cell: 3 (wedge, tetrahedra) or 4 (hex)
  int32_t tet;       // 1: each prism of a base triangle is split into 3 tetrahedra
  int32_t L;         // layers
  int32_t V;         // base vertices
  int32_t T;         // base cells
  int64_t n_cells;   // T * L
  int64_t n_dofs;    // 2 * V * (L + 1)
  const double4 *geo;      // [V] x, y, bed = s - H, H
  const double2 *sb;       // [V] s, beta
  const int64_t *colptr;   // [V + 1] first CSR entry of each vertex column's row block
  const int32_t *deg;      // [V] neighbouring columns including itself
  const int32_t *cells;    // [T * nv]
  const uint8_t *rank;     // [T * nv * nv] rank[a][b]: position of vertex b in a's neighbour list
  const double *sigma;     // [L + 1]
  // owner-computes work items: one per (vertex column v, base cell t containing v),
  // ordered by v; item i covers cell vc_idx[i] where v sits at local corner vc_pos[i]
  const int32_t *vc_ptr;   // [V + 1]
  const int32_t *vc_idx;   // [T * nv]
  const uint8_t *vc_pos;   // [T * nv]
  const int32_t *item_vtx; // [T * nv] vertex of each item
  const int32_t *slot_off; // [V] offset of v's rows inside its task's LDS level window
  const uint32_t *item_rank; // [T * nv] per item, 8 bits per corner: its rank in the
                             // item vertex's neighbour list
  double rho_g;            // rho * g
  double visc_pref;        // 1/2 A^(-1/n)
  double visc_exp;         // (1 - n) / (2 n)
  double n_glen;
  double A;
  double eps0_sq;
};

}  // namespace fo

struct fo_mesh {
  fo::MeshView view;
  int32_t elem;
  int64_t nnz;
  // device allocations owned by the mesh
  double4 *geo = nullptr;
  double2 *sb = nullptr;
  int64_t *colptr = nullptr;
  int32_t *deg = nullptr;
  int32_t *cells = nullptr;
  uint8_t *rank = nullptr;
  double *sigma = nullptr;
  int32_t *nbr_ptr = nullptr;   // [V + 1] sorted neighbour lists (incl. self)
  int32_t *nbr_idx = nullptr;
  int32_t *self_rank = nullptr; // [V] position of each vertex in its own neighbour list
  int32_t *vc_ptr = nullptr;    // [V + 1] base cells around each vertex
  int32_t *vc_idx = nullptr;
  uint8_t *vc_pos = nullptr;
  int32_t *item_vtx = nullptr;
  int32_t *slot_off = nullptr;
  uint32_t *item_rank = nullptr;
  // ocean fronts: the vertices on a front and, per front vertex, level and component, the
  // residual load of the fronts on that node (added after the cell assembly); NULL without
  int32_t n_front = 0;
  int32_t *front_vtx = nullptr;   // [n_front]
  double *front_load = nullptr;   // [n_front][L + 1][2]
  int4 *tasks = nullptr;        // [n_tasks] {member, v_begin, v_end, item_begin}
  int32_t n_tasks = 0;
  std::vector<int4> tasks_host; // host copy, for building ensembles
  int32_t max_slot = 0;         // largest LDS level window (entries) over tasks
  int32_t max_task_verts = 0;
  int64_t *rowptr = nullptr;    // [n_dofs + 1]
  int32_t *colidx = nullptr;    // [nnz]
  int device = 0;
  // optional kernel timing (fo_profile_enable / fo_profile_read)
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t n_recorded = 0;
};

namespace fo {
// One member of a batched ensemble launch: its mesh view, outputs and LDS window sizes.
struct EnsembleMember {
  MeshView view;
  const double *U;
  double *R;
  void *J;
  int32_t max_slot;
  int32_t max_tv;
};

struct EnsembleLaunch {
  const EnsembleMember *members;   // device [n_members]
  const int4 *tasks;               // device [n_tasks], .x = member index
  int32_t n_tasks;
  int *counter;                    // device work counter (16 bytes)
  int32_t nv;
  bool tet;
  bool all_n3;
  int32_t max_slot, max_tv;
  int32_t n_cu;
  int device;
};

fo_status launch_ensemble(const EnsembleLaunch &E, int dtype, int kind, bool want_jac, hipStream_t s);

// Ocean-front loads of a mesh description (fo_front.cpp): the vertices on a front and, per
// front vertex, level and component, the residual load.  Empty without fronts.
fo_status build_front_loads(const fo_mesh_desc *d, const std::vector<double> &sigma,
                            std::vector<int32_t> &vtx, std::vector<double> &load);

// Kernel launchers (fo_assemble.hip, fo_mesh_kernels.hip)
fo_status launch_pattern(const fo_mesh *m, hipStream_t s);
fo_status launch_assemble(const fo_mesh *m, const double *U, double *R, void *J, int dtype,
                          int kind, bool want_jac, hipStream_t s);
// the cell assembly alone (launch_assemble adds the ocean-front loads after it)
fo_status launch_assemble_cells(const fo_mesh *m, const double *U, double *R, void *J, int dtype,
                                int kind, bool want_jac, hipStream_t s);
fo_status launch_front_add(const MeshView &m, int32_t n_front, const int32_t *vtx, const double *load, double *R,
                           hipStream_t s);
fo_status launch_sia(const fo_mesh *m, double *U, hipStream_t s);
fo_status launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// learned initial guess (fo_learned.hip), shared with fo_newton_solve's FO_INIT_LEARNED
size_t learned_workspace_bytes(const fo_mesh *m);
fo_status learned_guess(const fo_mesh *m, const float *params, const float *norm, double *U, int32_t fallback,
                        int32_t sweeps, void *ws, size_t ws_bytes, int32_t *used_network,
                        int32_t *n_residuals, hipStream_t s);
// kernel timing brackets (no-ops unless profiling is enabled on the mesh)
fo_status profile_begin(const fo_mesh *m, hipStream_t s);
fo_status profile_end(const fo_mesh *m, hipStream_t s);
}  // namespace fo
