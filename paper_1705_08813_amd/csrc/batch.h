// Batched launches over many independent meshes (the serving path): the
// descriptors of up to K meshes (or mesh levels) travel by value in the
// kernel arguments of one launch, the workgroups of the launch dealt to
// them in order; larger batches take ceil(n / K) launches.  Segment s owns
// the blocks [blk0_s, blk0_{s+1}); blk0_0 = 0.  A mesh's segment runs the
// same compiled code in every launch it appears in, so its results do not
// depend on the other segments of the launch or on the batch.
#pragma once

#include "kern_common.h"

namespace dgwm {

// What the Poisson kernel does with y = A p at each output entry (solver fusion):
//   kPlain: y = A p
//   kResid: r = b - A p
//   kCheb:  v = c1 (p - zprev) + c2 dinv (b - A p), zout = p + v: one step
//           of the Chebyshev recurrence, whose previous iterate zprev is read
//           from zout before it is overwritten (c1 = 0: not read); zout must
//           not alias p
//   kChebFirst: the same step from the first iterate p = c0 dinv b (zprev =
//           0), which the kernel forms from b as it loads it (the input
//           pointer is b); p itself is written to z1 for the next step
enum PoiEpiKind { kPlain = 0, kResid = 1, kCheb = 2, kChebFirst = 3 };
template <typename T>
struct PoiEpi {
  int kind;
  const T* b;
  const T* dinv;
  T* z1;
  T* zout;
  T c1, c2, c0;
};

// Multigrid transfer geometry between a fine level and the next coarser one.
struct Tr {
  int nfx, nfy, nfz;   // fine level size
  int ncx, ncy, ncz;   // coarse level size
  int cx, cy, cz;
  const double* hyf;   // fine heights
};

// One mesh level of a batched Poisson launch (same degree and epilogue kind
// for every segment of a launch).
template <typename T>
struct PoiSeg {
  MeshDev M;
  const T* p;
  T* y;
  PoiEpi<T> E;
  int64_t ncell;
  int64_t blk0;
};

// One transfer of a batched restriction (out = P^T in) or prolongation
// (out = add + P in).
template <typename T>
struct TrSeg {
  Tr tr;
  const T* in;
  const T* add;
  T* out;
  int64_t ncc;
  int64_t blk0;
};

// x = B b with one mesh's dense coarsest-level inverse (n x n).
template <typename T>
struct DenseSeg {
  const T* B;
  const T* b;
  T* x;
  int64_t n;
  int64_t blk0;
};

// Segments per launch (kernel arguments stay below 4 KiB).
constexpr int kPoiSegs = 8, kTrSegs = 16, kDenseSegs = 32;
template <typename S, int K>
struct SegArr {
  S s[K];
  int n;
};

// Segment that owns block `bid` (segments sorted by blk0).
template <typename S, int K>
__device__ __forceinline__ int find_seg(const SegArr<S, K>& a, int64_t bid) {
  int lo = 0, hi = a.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.s[mid].blk0 <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Host side: descriptors of one mesh level, workgroup counts, batched launchers.
MeshDev poisson_meshdev(const dg_mesh* m, int l);
Tr mg_transfer_geometry(const dg_mesh* m, int l);
int poisson_cells_per_block(int np);
// the transfer kernel family a level pair uses and its coarse cells per workgroup
bool mg_full_transfer(const dg_mesh* m, int l);
int mg_cells_per_block(int np, bool full);
int dense_rows_per_block();

// The launchers take host arrays of segments (blk0 is filled in per launch)
// of one degree (and transfer family) and split them into launches of at
// most K segments.
template <typename T>
int launch_poisson_batched(int np, int kind, const PoiSeg<T>* segs, int nseg, hipStream_t s);
template <typename T>
int launch_mg_restrict_batched(int np, bool full, const TrSeg<T>* segs, int nseg, hipStream_t s);
template <typename T>
int launch_mg_prolong_batched(int np, bool full, const TrSeg<T>* segs, int nseg, hipStream_t s);
template <typename T>
int launch_dense_batched(const DenseSeg<T>* segs, int nseg, hipStream_t s);

}  // namespace dgwm
