// Cell-tile sort of the electron SoA (counting sort, every few steps).
//
// Electrons are keyed by the index of their spatial tile (Morton order over
// the bits all axes share, the longer axes' extra bits above); absorbed
// electrons get the largest key and end up behind the live ones (their last
// state is kept for read-back, they are never pushed again).  After a sort a
// contiguous chunk of electrons covers a compact box of cells, which is what
// lets the step kernel stage fields and accumulate currents in LDS.
//
// Passes: key + histogram (one atomic per distinct key in a workgroup), a two-pass exclusive
// scan of the tile counts, scatter into the second SoA buffer
// (order inside a tile is arbitrary; nothing downstream depends on it: the
// current is summed in fixed point and Philox streams follow the electron id).
//
// Absorbed electrons never change again, so a sort covers only the range that
// was live after the previous sort, [0, n_old): its live electrons go to the
// tiles and the ones absorbed since then to [n_new, n_old).  The older dead
// tail [n_old, N) is already in place in the destination buffer except for
// the stretch that died during the previous interval, [n_old, n_prev), which
// the scatter copies across to the same indices.  Counter words: n[0] live count (read by the step
// kernel), n[1] the count being built, n[2] the live count before the last
// sort.
#include <algorithm>
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

// Workgroup-level aggregation of equal keys: an LDS hash table (open
// addressing, twice as many slots as threads) counts the electrons of each
// distinct tile in the workgroup, so each tile costs one global atomic per
// workgroup however its electrons are ordered.
constexpr int kHash = 2 * kBlock;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

__device__ inline int hash_slot(uint32_t key) { return (int)((key * 2654435761u) >> 23) & (kHash - 1); }

// Add n electrons of key to the workgroup's table; returns its slot and,
// through before, the key's count before the addition.  (At most kBlock
// distinct keys in 2 kBlock slots: the probe always ends.)
__device__ inline int hash_add(uint32_t* hkey, uint32_t* hcnt, uint32_t key, uint32_t n,
                               uint32_t& before) {
  int h = hash_slot(key);
  for (;;) {
    const uint32_t prev = atomicCAS(&hkey[h], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      before = atomicAdd(&hcnt[h], n);
      return h;
    }
    h = (h + 1) & (kHash - 1);
  }
}

// The lanes of the wave that are active and hold this lane's key: one pass
// per distinct key of the wave.  A wave of a tile-sorted array nearly always
// holds one or two tiles, so its electrons enter the table with one or two
// LDS atomics instead of one per electron (same-address LDS atomics of a
// whole wave serialise).  Called by every lane of the wave.
__device__ inline uint64_t same_key_lanes(uint32_t key, bool active) {
  uint64_t todo = __ballot(active);
  uint64_t mine = 0ull;
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
    const bool eq = active && key == lk;
    const uint64_t m = __ballot(eq);
    if (eq) mine = m;
    todo &= ~m;
  }
  return mine;
}

// number of the set bits of mask below this lane
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_sort_key(SortArgs A) {
  __shared__ uint32_t hkey[kHash], hcnt[kHash];
  const int t = threadIdx.x;
  for (int i = t; i < kHash; i += kBlock) { hkey[i] = kEmpty; hcnt[i] = 0u; }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * kBlock + t;
  // id and position loaded together (every e < N is in bounds), before the
  // live count is known, so their latencies overlap
  uint32_t idv = kDead;
  int qv[3] = {0, 0, 0};
  R xv[3] = {R(0), R(0), R(0)};
  if (e < A.N) {
    idv = A.id[e];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= A.dims) break;
      if constexpr (sizeof(R) == 4) qv[a] = ((const int*)A.x[a])[e];
      else xv[a] = ((const R*)A.x[a])[e];
    }
  }
  const bool valid = e < (int64_t)A.n_active[0];
  uint32_t key = A.nkeys - 1;  // absorbed electrons: last bucket
  if (valid) {
    if (!(idv & kDead)) {
      uint32_t tt[3] = {0u, 0u, 0u};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a >= A.dims) break;
        int c;
        if constexpr (sizeof(R) == 4) c = qv[a] >> A.fb[a];  // fixed point
        else c = (int)floor(xv[a] * A.idx[a]);
        c = c < 0 ? 0 : (c >= A.n[a] ? A.n[a] - 1 : c);
        tt[a] = (uint32_t)(c / A.tile[a]);
      }
      if (A.dims == 1) {
        key = tt[0];
      } else {
        const uint32_t lm = (1u << A.mbits) - 1u;
        const uint32_t hi = (tt[0] >> A.mbits) | ((tt[1] >> A.mbits) << A.hb[0]) |
                            ((tt[2] >> A.mbits) << (A.hb[0] + A.hb[1]));
        if (A.dims == 2) key = (hi << (2 * A.mbits)) | spread2(tt[0] & lm) | (spread2(tt[1] & lm) << 1);
        else key = (hi << (3 * A.mbits)) | spread3(tt[0] & lm) | (spread3(tt[1] & lm) << 1) |
                   (spread3(tt[2] & lm) << 2);
      }
    }
    A.key[e] = key;
  }
  const uint64_t mine = same_key_lanes(key, valid);
  if (valid && lanes_below(mine) == 0u) {  // the first lane of each key counts its lanes
    uint32_t before;
    hash_add(hkey, hcnt, key, (uint32_t)__popcll(mine), before);
  }
  __syncthreads();
  for (int i = t; i < kHash; i += kBlock)
    if (hkey[i] != kEmpty) atomicAdd(A.count + hkey[i], hcnt[i]);
}

// Exclusive scan of count[0..nkeys) into offset and cursor, in two passes:
// segments of kSeg keys per workgroup, then a fix-up in which each
// workgroup adds the sum of the totals of the segments before its own.
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

__global__ __launch_bounds__(kBlock) void k_scan_fixup(SortArgs A, const uint32_t* btot) {
  __shared__ uint32_t part[kBlock / 64];
  const int64_t k0 = (int64_t)blockIdx.x * kSeg;
  uint32_t s = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kBlock) s += btot[b];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < kBlock / 64; ++w) add += part[w];
  for (int q = threadIdx.x; q < kSeg; q += kBlock) {
    const int64_t k = k0 + q;
    if (k < A.nkeys) {
      const uint32_t o = A.offset[k] + add;
      A.offset[k] = o;
      A.cursor[k] = o;
      // live electrons = everything before the absorbed bucket (the last key)
      if (k == A.nkeys - 1) A.n_active[1] = o;
    }
  }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(SortArgs A) {
  __shared__ uint32_t hkey[kHash], hcnt[kHash];
  const int t = threadIdx.x;
  for (int i = t; i < kHash; i += kBlock) { hkey[i] = kEmpty; hcnt[i] = 0u; }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * kBlock + t;
  // the electron's state is loaded up front (every e < N is in bounds), so its
  // latency overlaps the ranking and the cursor atomics
  R xv[3] = {R(0), R(0), R(0)}, pv[3] = {R(0), R(0), R(0)};
  double tv = 0.0, tbv = 0.0, wv = 0.0;
  uint32_t idv = 0u, kv = 0u;
  if (e < A.N) {
    kv = A.key[e];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < A.dims) xv[a] = ((const R*)A.x[a])[e];
      pv[a] = ((const R*)A.p[a])[e];
    }
    tv = A.tau[e];
    if (A.taub) tbv = A.taub[e];
    wv = A.w[e];
    idv = A.id[e];
  }
  const bool valid = e < (int64_t)A.n_active[0];
  // rank among the workgroup's electrons of the same key: the wave's range
  // for the key (taken by its first lane) plus the lanes of the key below
  const uint64_t mine = same_key_lanes(kv, valid);
  const int leader = valid ? __builtin_ctzll(mine) : (int)__lane_id();
  int h = 0;
  uint32_t before = 0u;
  if (valid && (int)__lane_id() == leader) h = hash_add(hkey, hcnt, kv, (uint32_t)__popcll(mine), before);
  h = __shfl(h, leader, 64);
  const uint32_t rank = (uint32_t)__shfl((int)before, leader, 64) + lanes_below(mine);
  __syncthreads();
  // one cursor atomic per distinct key of the workgroup; the slot's count is
  // replaced by the base of the workgroup's range for that key
  for (int i = t; i < kHash; i += kBlock)
    if (hkey[i] != kEmpty) hcnt[i] = atomicAdd(A.cursor + hkey[i], hcnt[i]);
  __syncthreads();
  // electrons of the dead stretch [n_old, n_prev) keep their index (they
  // were absorbed before the last sort and are no longer in the ranked range)
  const bool tail = !valid && e < (int64_t)A.n_active[2];
  if (!valid && !tail) return;
  const int64_t d = valid ? (int64_t)(hcnt[h] + rank) : e;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < A.dims) ((R*)A.x2[a])[d] = xv[a];
    ((R*)A.p2[a])[d] = pv[a];
  }
  A.tau2[d] = tv;
  if (A.taub) A.taub2[d] = tbv;
  A.w2[d] = wv;
  A.id2[d] = idv;
}

__global__ void k_sort_commit(uint32_t* n) {
  n[2] = n[0];
  n[0] = n[1];
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
  hipLaunchKernelGGL(k_scan_fixup, dim3(nseg), dim3(kBlock), 0, s, A, btot);
  if (fp32) hipLaunchKernelGGL(k_sort_scatter<float>, dim3(blocks), dim3(kBlock), 0, s, A);
  else hipLaunchKernelGGL(k_sort_scatter<double>, dim3(blocks), dim3(kBlock), 0, s, A);
  hipLaunchKernelGGL(k_sort_commit, dim3(1), dim3(1), 0, s, A.n_active);
}

}  // namespace pic
