// Cell-tile sort of the electron SoA (counting sort, every few steps).
//
// Electrons are keyed by the Morton index of their spatial tile; absorbed
// electrons get the largest key and end up behind the live ones (their last
// state is kept for read-back, they are never pushed again).  After a sort a
// contiguous chunk of electrons covers a compact box of cells, which is what
// lets the step kernel stage fields and accumulate currents in LDS.
//
// Passes: key + histogram (one atomic per run of equal keys in a wave), a three-pass exclusive
// scan of the tile counts, scatter into the second SoA buffer
// (order inside a tile is arbitrary; nothing downstream depends on it: the
// current is summed in fixed point and Philox streams follow the electron id).
#include "pic_internal.hpp"

namespace pic {

__device__ inline uint32_t spread2(uint32_t v) {  // 16 bits -> even bit positions
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ inline uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Runs of equal keys inside a wave (the input is mostly sorted already):
// first lane of the run and its length, so one atomic serves the whole run.
struct Run {
  int start, len;
};
__device__ inline Run wave_run(uint32_t key, bool valid) {
  const int lane = (int)__lane_id();
  const uint32_t prev = __shfl_up(key, 1u, 64);
  const bool head = valid && (lane == 0 || prev != key);
  const unsigned long long heads = __ballot(head);
  const unsigned long long valids = __ballot(valid);
  const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
  const int start = 63 - __clzll(heads & upto);
  const unsigned long long after = start == 63 ? 0ull : (heads & ~((1ull << (start + 1)) - 1ull));
  const int end = after ? __ffsll((long long)after) - 1 : __popcll(valids);
  return Run{start, end - start};
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_sort_key(SortArgs A) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = e < A.N;
  uint32_t key = A.nkeys - 1;  // absorbed electrons: last bucket
  if (valid && !(A.id[e] & kDead)) {
    uint32_t t[3] = {0u, 0u, 0u};
    for (int a = 0; a < A.dims; ++a) {
      int c;
      if constexpr (sizeof(R) == 4) c = ((const int*)A.x[a])[e] >> A.fb[a];  // fixed point
      else c = (int)floor(((const R*)A.x[a])[e] * A.idx[a]);
      c = c < 0 ? 0 : (c >= A.n[a] ? A.n[a] - 1 : c);
      t[a] = (uint32_t)(c / A.tile[a]);
    }
    if (A.dims == 1) key = t[0];
    else if (A.dims == 2) key = spread2(t[0]) | (spread2(t[1]) << 1);
    else key = spread3(t[0]) | (spread3(t[1]) << 1) | (spread3(t[2]) << 2);
  }
  const Run r = wave_run(key, valid);
  if (!valid) return;
  A.key[e] = key;
  if ((int)__lane_id() == r.start) atomicAdd(A.count + key, (uint32_t)r.len);
}

// Exclusive scan of count[0..nkeys) into offset and cursor, in three passes:
// segments of kSeg keys per workgroup, the segment totals, then the fix-up.
constexpr int kSeg = 4096;                 // 256 threads x 16 keys
constexpr int kPerThread = kSeg / kBlock;

__global__ __launch_bounds__(kBlock) void k_scan_segments(SortArgs A, uint32_t* btot) {
  __shared__ uint32_t part[kBlock];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kSeg + (int64_t)t * kPerThread;
  uint32_t v[kPerThread];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t k = base + q;
    v[q] = k < A.nkeys ? A.count[k] : 0u;
    s += v[q];
  }
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {   // inclusive scan of the thread sums
    const uint32_t u = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  uint32_t run = t == 0 ? 0u : part[t - 1];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t k = base + q;
    if (k < A.nkeys) {
      A.offset[k] = run;
      A.count[k] = 0u;  // ready for the next sort
    }
    run += v[q];
  }
  if (t == kBlock - 1) btot[blockIdx.x] = part[t];
}

__global__ __launch_bounds__(1024) void k_scan_totals(uint32_t* btot, int nseg) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int per = (nseg + 1023) / 1024;
  const int lo = t * per, hi = min(nseg, lo + per);
  uint32_t s = 0;
  for (int k = lo; k < hi; ++k) s += btot[k];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t u = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  uint32_t run = t == 0 ? 0u : part[t - 1];
  for (int k = lo; k < hi; ++k) {
    const uint32_t c = btot[k];
    btot[k] = run;
    run += c;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_fixup(SortArgs A, const uint32_t* btot) {
  const int64_t k0 = (int64_t)blockIdx.x * kSeg;
  const uint32_t add = btot[blockIdx.x];
  for (int q = threadIdx.x; q < kSeg; q += kBlock) {
    const int64_t k = k0 + q;
    if (k < A.nkeys) {
      const uint32_t o = A.offset[k] + add;
      A.offset[k] = o;
      A.cursor[k] = o;
      // live electrons = everything before the absorbed bucket (the last key)
      if (k == A.nkeys - 1) *A.n_active = o;
    }
  }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(SortArgs A) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = e < A.N;
  const uint32_t key = valid ? A.key[e] : 0xFFFFFFFFu;
  const Run r = wave_run(key, valid);
  const int lane = (int)__lane_id();
  uint32_t base = 0;
  if (valid && lane == r.start) base = atomicAdd(A.cursor + key, (uint32_t)r.len);
  base = __shfl(base, r.start, 64);
  if (!valid) return;
  const uint32_t d = base + (uint32_t)(lane - r.start);
  for (int a = 0; a < A.dims; ++a) ((R*)A.x2[a])[d] = ((const R*)A.x[a])[e];
  for (int a = 0; a < 3; ++a) ((R*)A.p2[a])[d] = ((const R*)A.p[a])[e];
  A.tau2[d] = A.tau[e];
  A.w2[d] = A.w[e];
  A.id2[d] = A.id[e];
}

int sort_scratch_words(uint32_t nkeys) { return (int)(((int64_t)nkeys + kSeg - 1) / kSeg); }

void launch_sort(const SortArgs& A, bool fp32, hipStream_t s) {
  if (A.N <= 0) return;
  const unsigned blocks = (unsigned)((A.N + kBlock - 1) / kBlock);
  if (fp32) hipLaunchKernelGGL(k_sort_key<float>, dim3(blocks), dim3(kBlock), 0, s, A);
  else hipLaunchKernelGGL(k_sort_key<double>, dim3(blocks), dim3(kBlock), 0, s, A);
  const int nseg = (int)(((int64_t)A.nkeys + kSeg - 1) / kSeg);
  uint32_t* btot = A.cursor + A.nkeys;  // nseg scratch words after the cursors
  hipLaunchKernelGGL(k_scan_segments, dim3(nseg), dim3(kBlock), 0, s, A, btot);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, btot, nseg);
  hipLaunchKernelGGL(k_scan_fixup, dim3(nseg), dim3(kBlock), 0, s, A, btot);
  if (fp32) hipLaunchKernelGGL(k_sort_scatter<float>, dim3(blocks), dim3(kBlock), 0, s, A);
  else hipLaunchKernelGGL(k_sort_scatter<double>, dim3(blocks), dim3(kBlock), 0, s, A);
}

}  // namespace pic
