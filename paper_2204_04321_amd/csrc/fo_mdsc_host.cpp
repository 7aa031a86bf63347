// Host side of the two-level column semicoarsening preconditioner: aggregation of the plane
// graph and the tables that the device kernels use to restrict, prolong and form the Galerkin
// operators (arXiv:2204.04321 Sec. 3.3: aggregation AMG on the plane once the extruded mesh
// is collapsed to one layer).
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "fo_mdsc.h"

namespace fo {

constexpr int kIsolatedGroup = 8;

// Pass 1, vertices in index order: an unassigned vertex whose other neighbours are all
// unassigned roots an aggregate of itself and those neighbours; an isolated vertex joins the
// open group of isolated vertices (a new group every kIsolatedGroup members).  Pass 2: each
// vertex still unassigned joins the aggregate of its lowest-numbered neighbour assigned in
// pass 1 (one exists: when pass 1 skipped it, some neighbour was already assigned).
int32_t aggregate_graph(const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                        std::vector<int32_t> &agg) {
  const int32_t n = int32_t(ptr.size()) - 1;
  agg.assign(size_t(n), -1);
  int32_t n_agg = 0, open_group = -1, open_count = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (agg[v] >= 0) continue;
    bool has_other = false, all_free = true;
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e) {
      const int32_t w = idx[e];
      if (w == v) continue;
      has_other = true;
      if (agg[w] >= 0) { all_free = false; break; }
    }
    if (!has_other) {
      if (open_group < 0 || open_count == kIsolatedGroup) { open_group = n_agg++; open_count = 0; }
      agg[v] = open_group;
      ++open_count;
      continue;
    }
    if (!all_free) continue;
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e) agg[idx[e]] = n_agg;
    ++n_agg;
  }
  const std::vector<int32_t> pass1 = agg;
  for (int32_t v = 0; v < n; ++v) {
    if (agg[v] >= 0) continue;
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e)   // sorted: the first hit is the lowest
      if (pass1[idx[e]] >= 0) { agg[v] = pass1[idx[e]]; break; }
  }
  return n_agg;
}

// Graph of the aggregates (sorted lists with the aggregate itself), the members of each
// aggregate in ascending order, and for every block of the coarse graph the blocks of the fine
// graph that sum into it (ascending, so the Galerkin sums run in a fixed order).
void coarse_tables(const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx, const std::vector<int32_t> &agg,
                   int32_t n_agg, PlaneTables &t) {
  const int32_t n = int32_t(ptr.size()) - 1;
  std::vector<std::vector<int32_t>> rows(static_cast<size_t>(n_agg));
  for (int32_t v = 0; v < n; ++v)
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e) rows[agg[v]].push_back(agg[idx[e]]);
  t.cptr.assign(size_t(n_agg) + 1, 0);
  t.cidx.clear();
  for (int32_t a = 0; a < n_agg; ++a) {
    auto &r = rows[a];
    r.push_back(a);
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    t.cidx.insert(t.cidx.end(), r.begin(), r.end());
    t.cptr[a + 1] = int32_t(t.cidx.size());
  }
  t.mptr.assign(size_t(n_agg) + 1, 0);
  for (int32_t v = 0; v < n; ++v) t.mptr[agg[v] + 1]++;
  for (int32_t a = 0; a < n_agg; ++a) t.mptr[a + 1] += t.mptr[a];
  t.midx.assign(size_t(n), 0);
  {
    std::vector<int32_t> fill(t.mptr.begin(), t.mptr.end() - 1);
    for (int32_t v = 0; v < n; ++v) t.midx[fill[agg[v]]++] = v;
  }
  const int32_t nnz_f = ptr[n], nnz_c = t.cptr[n_agg];
  std::vector<int32_t> target(static_cast<size_t>(nnz_f));
  for (int32_t v = 0; v < n; ++v) {
    const int32_t a = agg[v];
    const auto b0 = t.cidx.begin() + t.cptr[a], b1 = t.cidx.begin() + t.cptr[a + 1];
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e)
      target[e] = int32_t(std::lower_bound(b0, b1, agg[idx[e]]) - t.cidx.begin());
  }
  t.gptr.assign(size_t(nnz_c) + 1, 0);
  for (int32_t e = 0; e < nnz_f; ++e) t.gptr[target[e] + 1]++;
  for (int32_t c = 0; c < nnz_c; ++c) t.gptr[c + 1] += t.gptr[c];
  t.gidx.assign(size_t(nnz_f), 0);
  std::vector<int32_t> fill(t.gptr.begin(), t.gptr.end() - 1);
  for (int32_t e = 0; e < nnz_f; ++e) t.gidx[fill[target[e]]++] = e;
}

bool graph_ok(int32_t n, const int32_t *ptr, const int32_t *idx, std::string &why) {
  if (n < 1 || !ptr || !idx) { why = "empty graph or NULL lists"; return false; }
  if (ptr[0] != 0) { why = "ptr[0] must be 0"; return false; }
  for (int32_t v = 0; v < n; ++v) {
    if (ptr[v + 1] <= ptr[v]) { why = "vertex " + std::to_string(v) + " has an empty list"; return false; }
    bool self = false;
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e) {
      if (idx[e] < 0 || idx[e] >= n) { why = "neighbour index out of range"; return false; }
      if (e > ptr[v] && idx[e] <= idx[e - 1]) { why = "lists must be sorted without repeats"; return false; }
      self = self || idx[e] == v;
    }
    if (!self) { why = "vertex " + std::to_string(v) + " is missing from its own list"; return false; }
  }
  return true;
}

}  // namespace fo

extern "C" fo_status fo_mdsc_aggregate_graph(int32_t n, const int32_t *ptr, const int32_t *idx, int32_t *agg,
                                             int32_t *n_agg) {
  std::string why;
  if (!agg || !n_agg) return fo::fail(FO_EINVAL, "fo_mdsc_aggregate_graph: NULL output");
  if (!fo::graph_ok(n, ptr, idx, why)) return fo::fail(FO_EINVAL, "fo_mdsc_aggregate_graph: " + why);
  std::vector<int32_t> p(ptr, ptr + n + 1), ix(idx, idx + ptr[n]), a;
  *n_agg = fo::aggregate_graph(p, ix, a);
  std::copy(a.begin(), a.end(), agg);
  return FO_OK;
}
