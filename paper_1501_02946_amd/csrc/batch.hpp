// Batched execution: many independent problems, one persistent launch per
// pipeline stage. Every stage has a work list of (problem, block) items in
// scheduling order (largest problems first); resident workgroups take items
// from an atomic queue until the list is exhausted, so uneven problem sizes
// balance across the chip. Each item runs the same device body as the
// single-problem kernel, so the arithmetic of a problem is unchanged and its
// result does not depend on which workgroup computed it.
#pragma once
#include "kparams.hpp"

namespace nedner {

struct BatchProb {
  KP kp;
  const void* g;  // data of this problem (written before each execute)
  void* out;      // volume of this problem (written before each execute)
  void* b0;       // workspace slice, buffer 0
  void* b1;       // workspace slice, buffer 1
};

struct WorkList {
  const int2* items;  // (problem, block) pairs
  int total;
  int* counter;       // queue head; zero when the launch starts
};

template <class F>
__device__ __forceinline__ void work_loop(const WorkList& wl, F&& f) {
  __shared__ int s_item;
  for (;;) {
    __syncthreads();  // the previous item is finished before LDS and s_item are reused
    if (threadIdx.x == 0) s_item = atomicAdd(wl.counter, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= wl.total) break;
    const int2 w = wl.items[it];
    f(w.x, w.y);
  }
}

// Blocks (items) one problem contributes to each forward stage.
enum Stage { ST_SPREAD = 0, ST_LAT_A, ST_LAT_B, ST_COLUMN, ST_PASS_C, ST_PASS_D, ST_COUNT };

// Up to 64 problems' data and volume pointers, written into the device
// problem table by one small kernel on the execute stream.
struct PtrChunk {
  int first, n;
  const void* g[64];
  void* out[64];
};

hipError_t launch_batch_prepare(BatchProb* bp, const PtrChunk& c, int* counters, int ncounters,
                                hipStream_t s);
hipError_t launch_spread_many(const KP& p0, const BatchProb* bp, const WorkList& wl, int vec,
                              hipStream_t s);
hipError_t launch_pass_many(const KP& p0, int stage, const BatchProb* bp, const WorkList& wl,
                            size_t smem, hipStream_t s);
hipError_t launch_column_many(const KP& p0, const BatchProb* bp, const WorkList& wl, int cpw,
                              size_t smem, hipStream_t s);
size_t column_wave_bytes_host(const KP& p);
int column_wpc_host(const KP& p);
int column_ppt_host(const KP& p);
size_t column_shared_bytes_host(const KP& p);

}  // namespace nedner
