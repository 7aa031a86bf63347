// Internal declarations of the two-level column semicoarsening preconditioner.
#pragma once

#include <string>
#include <vector>

#include "fo_internal.h"

namespace fo {

constexpr int kMdscCoarsestMax = 64;      // plane vertices solved by the dense inverse
constexpr int kMdscMaxLevels = 24;

// Host tables that link one plane level to the next (coarser) one.
struct PlaneTables {
  std::vector<int32_t> cptr, cidx;   // graph of the aggregates
  std::vector<int32_t> mptr, midx;   // members of each aggregate
  std::vector<int32_t> gptr, gidx;   // per coarse block: the fine blocks summed into it
};

int32_t aggregate_graph(const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx, std::vector<int32_t> &agg);
void coarse_tables(const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx, const std::vector<int32_t> &agg,
                   int32_t n_agg, PlaneTables &t);
bool graph_ok(int32_t n, const int32_t *ptr, const int32_t *idx, std::string &why);

// One plane level on the device.  Blocks are 2x2, stored [2 c + d] (row component c, column
// component d); vectors hold 2 values per vertex.
struct PlaneLevel {
  int32_t n = 0, nnzb = 0;
  std::vector<int32_t> ptr_h, idx_h, agg_h;
  const int32_t *ptr = nullptr, *idx = nullptr;   // level 0: the mesh's neighbour lists
  int32_t *own_ptr = nullptr, *own_idx = nullptr;
  int32_t *diag = nullptr;      // [n] index of each vertex's diagonal block
  double *A = nullptr;          // [4 nnzb]
  double *Dinv = nullptr;       // [4 n]
  double *bound = nullptr;      // [n] Gershgorin row bounds
  double *g = nullptr;          // [1] their maximum
  int32_t *agg = nullptr;       // [n] aggregate of each vertex (smoothed levels)
  int32_t *mptr = nullptr, *midx = nullptr;   // members of the next level's vertices
  int32_t *gptr = nullptr, *gidx = nullptr;   // Galerkin gather lists for the next level
  double *b = nullptr, *x = nullptr;          // [2 n] right-hand side and iterate
  double *x2 = nullptr, *d = nullptr;         // [2 n] degree-2 smoothing state (first level only)
};

// The device view of one plane level (what the V-cycle kernels read).
struct LevelDev {
  int32_t n;
  const int32_t *ptr, *idx, *agg, *mptr, *midx;
  const double *A, *Dinv, *g;
  double *b, *x, *x2, *d;
};

}  // namespace fo

struct fo_mdsc {
  const fo_mesh *mesh = nullptr;
  int device = 0;
  std::vector<fo::PlaneLevel> lv;   // lv.back() is the coarsest
  int32_t *blk_row = nullptr;       // [nnzb of level 0] row vertex of each block
  fo::LevelDev *lv_dev = nullptr;   // [levels] device copies of the level views
  float *fac = nullptr;             // column factors, the layout of the column preconditioner
  double *W = nullptr;              // [V][L+1][2][2] collapse weights (FP64, for the setup)
  float *W32 = nullptr;             // the same rounded to FP32 (restriction and prolongation)
  float *JP = nullptr;              // J P0 (FP32) by plane block e = (v, r): entry d of row q
                                    // of column v at (2 e + d) 2 (L+1) + q
  size_t jp_count = 0;
  double *Ainv = nullptr;           // coarsest inverse, row-major [nc][nc]
  int32_t *flag = nullptr;          // device status of the last setup
  int32_t *flag_host = nullptr;     // pinned
  bool ready = false;
};
