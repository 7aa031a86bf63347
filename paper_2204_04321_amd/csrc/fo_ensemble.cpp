// Batched ensembles: many extruded meshes (uneven sizes, their own beta, A, ...) assembled
// by one persistent launch that pulls (member, task) work items from a combined table.
#include <hip/hip_runtime.h>

#include <vector>

#include "fo_internal.h"

struct fo_ensemble {
  std::vector<const fo_mesh *> members;
  fo::EnsembleLaunch launch{};
  fo::EnsembleMember *dev_members = nullptr;
  int4 *dev_tasks = nullptr;
  int *dev_counter = nullptr;
  fo::EnsembleMember *staging = nullptr;   // pinned host copy of the member table
  hipEvent_t staged{};
  bool has_event = false;
};

using namespace fo;

static void free_ensemble(fo_ensemble *e) {
  if (!e) return;
  if (e->has_event) (void)hipEventDestroy(e->staged);
  if (e->dev_members) (void)hipFree(e->dev_members);
  if (e->dev_tasks) (void)hipFree(e->dev_tasks);
  if (e->dev_counter) (void)hipFree(e->dev_counter);
  if (e->staging) (void)hipHostFree(e->staging);
  delete e;
}

extern "C" fo_status fo_ensemble_create(const fo_mesh *const *members, int32_t n_members, void *stream,
                                        fo_ensemble **out) {
  if (!out) return fail(FO_EINVAL, "fo_ensemble_create: out is NULL");
  *out = nullptr;
  if (!members || n_members < 1) return fail(FO_EINVAL, "fo_ensemble_create: need at least one member");
  const int nv = members[0] ? members[0]->view.nv : 0;
  int64_t total = 0;
  bool all_n3 = true;
  int32_t max_slot = 0, max_tv = 0;
  for (int i = 0; i < n_members; ++i) {
    const fo_mesh *m = members[i];
    if (!m) return fail(FO_EINVAL, "fo_ensemble_create: NULL member");
    if (m->view.nv != nv || m->view.tet != members[0]->view.tet)
      return fail(FO_EINVAL, "fo_ensemble_create: members must share the element type");
    total += m->n_tasks;
    all_n3 = all_n3 && m->view.n_glen == 3.0;
    max_slot = std::max(max_slot, m->max_slot);
    max_tv = std::max(max_tv, m->max_task_verts);
  }
  if (total >= (int64_t(1) << 31)) return fail(FO_EINVAL, "fo_ensemble_create: too many work items");
  std::vector<int4> tasks;
  tasks.reserve(size_t(total));
  for (int i = 0; i < n_members; ++i)
    for (const int4 &t : members[i]->tasks_host) tasks.push_back(make_int4(i, t.y, t.z, t.w));

  fo_ensemble *e = new fo_ensemble();
  e->members.assign(members, members + n_members);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto bail = [&](fo_status st, const char *msg) { free_ensemble(e); return fail(st, msg); };
  if (hipMalloc(&e->dev_members, sizeof(EnsembleMember) * n_members) != hipSuccess ||
      hipMalloc(&e->dev_tasks, sizeof(int4) * tasks.size()) != hipSuccess ||
      hipMalloc(&e->dev_counter, 16) != hipSuccess)
    return bail(FO_ENOMEM, "fo_ensemble_create: device allocation failed");
  if (hipHostMalloc(reinterpret_cast<void **>(&e->staging), sizeof(EnsembleMember) * n_members) != hipSuccess)
    return bail(FO_ENOMEM, "fo_ensemble_create: pinned allocation failed");
  if (hipEventCreateWithFlags(&e->staged, hipEventDisableTiming) != hipSuccess)
    return bail(FO_EDEVICE, "fo_ensemble_create: event creation failed");
  e->has_event = true;
  if (hipMemcpyAsync(e->dev_tasks, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(FO_EDEVICE, "fo_ensemble_create: upload failed");
  int dev = 0, n_cu = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) n_cu = 1;
  EnsembleLaunch &L = e->launch;
  L.members = e->dev_members;
  L.tasks = e->dev_tasks;
  L.n_tasks = int32_t(tasks.size());
  L.counter = e->dev_counter;
  L.nv = nv;
  L.tet = members[0]->view.tet != 0;
  L.all_n3 = all_n3;
  L.max_slot = max_slot;
  L.max_tv = max_tv;
  L.n_cu = n_cu;
  L.device = dev;
  *out = e;
  return FO_OK;
}

extern "C" void fo_ensemble_destroy(fo_ensemble *e) { free_ensemble(e); }

extern "C" fo_status fo_ensemble_assemble(fo_ensemble *e, const double *const *U_dev, double *const *R_dev,
                                          void *const *J_dev, int32_t dtype, int32_t kind, void *stream) {
  if (!e || !U_dev) return fail(FO_EINVAL, "fo_ensemble_assemble: NULL argument");
  if (dtype != FO_F64 && dtype != FO_F32) return fail(FO_EINVAL, "fo_ensemble_assemble: bad dtype");
  if (kind != FO_JAC_NEWTON && kind != FO_JAC_PICARD) return fail(FO_EINVAL, "fo_ensemble_assemble: bad kind");
  const bool want_jac = J_dev != nullptr;
  const int n = int(e->members.size());
  // the previous call's member table must have reached the device before it is rewritten
  FO_HIP_TRY(hipEventSynchronize(e->staged));
  for (int i = 0; i < n; ++i) {
    const void *u = U_dev[i];
    void *r = R_dev ? R_dev[i] : nullptr;
    void *j = want_jac ? J_dev[i] : nullptr;
    if (!u || (want_jac && !j) || (!want_jac && !r))
      return fail(FO_EINVAL, "fo_ensemble_assemble: missing member buffer");
    if ((reinterpret_cast<uintptr_t>(u) & 15) || (reinterpret_cast<uintptr_t>(r) & 15) ||
        (reinterpret_cast<uintptr_t>(j) & 15))
      return fail(FO_EINVAL, "fo_ensemble_assemble: member buffers must be 16-byte aligned");
    EnsembleMember &m = e->staging[i];
    m.view = e->members[i]->view;
    m.U = static_cast<const double *>(u);
    m.R = static_cast<double *>(r);
    m.J = j;
    m.max_slot = e->members[i]->max_slot;
    m.max_tv = e->members[i]->max_task_verts;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  FO_HIP_TRY(hipMemcpyAsync(e->dev_members, e->staging, sizeof(EnsembleMember) * n, hipMemcpyHostToDevice, s));
  FO_HIP_TRY(hipEventRecord(e->staged, s));
  fo_status st = launch_ensemble(e->launch, dtype, kind, want_jac, s);
  if (st != FO_OK) return st;
  for (int i = 0; i < n; ++i) {   // members with ocean fronts: their memoised loads
    const fo_mesh *m = e->members[i];
    if (m->n_front > 0 && R_dev && R_dev[i] &&
        (st = launch_front_add(m->view, m->n_front, m->front_vtx, m->front_load, R_dev[i], s)) != FO_OK)
      return st;
  }
  return FO_OK;
}
