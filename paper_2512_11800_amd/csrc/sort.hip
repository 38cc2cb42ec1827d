// Device-wide exclusive scan and a stable LSD radix sort used to build the
// per-tile Gaussian lists. No depth sort is needed: the moment and quadrature
// passes are order independent (Sec. 3.3), so lists are ordered by tile only,
// and by entry index inside a tile (stable), which keeps results bitwise
// reproducible.
#include "kernels.h"

namespace mb {

constexpr int kItems = 8;                  // items per thread
constexpr int kChunk = kBlock * kItems;    // items per block

__device__ __forceinline__ int wave_inclusive_sum(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// exclusive prefix of v over the 256 threads of the block; *total gets the sum
__device__ __forceinline__ int block_exclusive_sum(int v, int* lds4, int* total) {
  int inc = wave_inclusive_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 63) lds4[wave] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    int s = lds4[w];
    off += (w < wave) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const int* in, int64_t n, int* sums) {
  int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    s += (i < n) ? in[i] : 0;
  }
  __shared__ int lds[4];
  int tot;
  block_exclusive_sum(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of `sums[0..m)` in place, total to *total
__global__ __launch_bounds__(256) void k_scan_top(int* sums, int64_t m, int* total) {
  int64_t per = (m + kBlock - 1) / kBlock;
  int64_t b0 = threadIdx.x * per;
  int s = 0;
  for (int64_t k = 0; k < per; ++k) {
    int64_t i = b0 + k;
    if (i < m) s += sums[i];
  }
  __shared__ int lds[4];
  int tot;
  int off = block_exclusive_sum(s, lds, &tot);
  for (int64_t k = 0; k < per; ++k) {
    int64_t i = b0 + k;
    if (i < m) {
      int v = sums[i];
      sums[i] = off;
      off += v;
    }
  }
  if (threadIdx.x == 0 && total != nullptr) *total = tot;
}

__global__ __launch_bounds__(256) void k_scan_down(const int* in, int* out, int64_t n, const int* sums) {
  int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
  int v[kItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    v[k] = (i < n) ? in[i] : 0;
    s += v[k];
  }
  __shared__ int lds[4];
  int tot;
  int off = block_exclusive_sum(s, lds, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = off;
    off += v[k];
  }
}

// Down-sweep that forms its block's offset itself: the sum of the block sums
// before it (fixed order), for at most kDirectBlocks blocks; block 0 also
// writes the total. Saves the single-block pass between the two sweeps.
constexpr int kDirectBlocks = 1024;

__global__ __launch_bounds__(256) void k_scan_down_direct(const int* in, int* out, int64_t n, const int* sums,
                                                          int nb, int* total) {
  __shared__ int lds[4];
  const int upto = total != nullptr && blockIdx.x == 0 ? nb : (int)blockIdx.x;
  int s = 0;
  for (int i = threadIdx.x; i < upto; i += kBlock) s += sums[i];
  int tot;
  block_exclusive_sum(s, lds, &tot);
  int before = tot;  // blocks [0, upto)
  if (blockIdx.x == 0) {
    if (total != nullptr && threadIdx.x == 0) *total = tot;
    before = 0;
  }
  int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x * kItems;
  int v[kItems];
  int t = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    v[k] = (i < n) ? in[i] : 0;
    t += v[k];
  }
  int off = block_exclusive_sum(t, lds, &tot) + before;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = off;
    off += v[k];
  }
}

size_t scan_tmp_ints(int64_t n) { return (size_t)((n + kChunk - 1) / kChunk) + 1; }

hipError_t launch_scan(const int* in, int* out, int64_t n, int* tmp, int* total, hipStream_t s) {
  int64_t nb = (n + kChunk - 1) / kChunk;
  if (nb == 0) {
    if (total) return hipMemsetAsync(total, 0, sizeof(int), s);
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tmp);
  if (nb <= kDirectBlocks) {
    hipLaunchKernelGGL(k_scan_down_direct, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, tmp, (int)nb,
                       total);
  } else {
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, tmp, nb, total);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, tmp);
  }
  return hipGetLastError();
}

// Item count of a launch sized for n_max items: *n_dev when the count lives
// on the device (clamped to n_max), else n_max.
__device__ __forceinline__ int64_t items_of(const int* n_dev, int64_t n_max) {
  return n_dev ? min((int64_t)max(*n_dev, 0), n_max) : n_max;
}

// ---------------------------------------------------------------------------
// Radix sort, 8-bit digits. Per pass: block histograms (digit-major), their
// exclusive scan, then a stable scatter in which every block walks its chunk
// in index order, 256 items per round, ranking equal digits inside a wave
// with ballots and across waves through LDS counters.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* keys, int64_t n_max, const int* n_dev,
                                                    int shift, int* hist, int nblocks) {
  const int64_t n = items_of(n_dev, n_max);
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kChunk;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* keys_in, const int* vals_in,
                                                       uint32_t* keys_out, int* vals_out, int64_t n_max,
                                                       const int* n_dev, int shift, const int* offsets,
                                                       int nblocks) {
  const int64_t n = items_of(n_dev, n_max);
  __shared__ int running[256];
  __shared__ int wave_cnt[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  running[tid] = offsets[(int64_t)tid * nblocks + blockIdx.x];
#pragma unroll
  for (int w = 0; w < 4; ++w) wave_cnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kChunk;
  for (int r = 0; r < kItems; ++r) {
    int64_t i = base + r * kBlock + tid;
    bool valid = i < n;
    uint32_t key = valid ? keys_in[i] : 0u;
    int val = valid ? (vals_in ? vals_in[i] : (int)i) : 0;  // no vals_in: the identity
    uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      bool b = (d >> bit) & 1u;
      uint64_t m = __ballot(b);
      peers &= b ? m : ~m;
    }
    int rank = __popcll(peers & lt);
    if (valid && rank == 0) wave_cnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = running[d] + rank;
#pragma unroll
      for (int w = 0; w < 4; ++w) pos += (w < wave) ? wave_cnt[w][d] : 0;
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    running[tid] += wave_cnt[0][tid] + wave_cnt[1][tid] + wave_cnt[2][tid] + wave_cnt[3][tid];
#pragma unroll
    for (int w = 0; w < 4; ++w) wave_cnt[w][tid] = 0;
    __syncthreads();
  }
}

size_t radix_tmp_ints(int64_t n) {
  int64_t nb = (n + kChunk - 1) / kChunk;
  return (size_t)(256 * nb) + scan_tmp_ints(256 * nb) + 1;
}

// one stable pass on digit (key >> shift) & 255
static hipError_t radix_pass(const uint32_t* kin, const int* vin, uint32_t* kout, int* vout, int64_t n,
                             const int* n_dev, int shift, int* tmp, hipStream_t s) {
  const int64_t nb = (n + kChunk - 1) / kChunk;
  int* hist = tmp;
  int* scan_tmp = tmp + 256 * nb;
  hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, n, n_dev, shift, hist, (int)nb);
  hipError_t e = launch_scan(hist, hist, 256 * nb, scan_tmp, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, vin, kout, vout, n, n_dev, shift,
                     hist, (int)nb);
  return hipGetLastError();
}

hipError_t launch_radix_sort(uint32_t* keys_a, int* vals_a, uint32_t* keys_b, int* vals_b, int64_t n,
                             const int* n_dev, int bits, int* tmp, hipStream_t s, bool identity_vals) {
  const int passes = (bits + 7) / 8;
  if (n <= 0 || passes <= 0) return hipSuccess;
  uint32_t* kbuf[2] = {keys_a, keys_b};
  int* vbuf[2] = {vals_a, vals_b};
  int cur = 0;  // buffer holding the input of the next pass
  for (int p = 0; p < passes; ++p) {
    const int* vin = (p == 0 && identity_vals) ? nullptr : vbuf[cur];
    hipError_t e = radix_pass(kbuf[cur], vin, kbuf[cur ^ 1], vbuf[cur ^ 1], n, n_dev, 8 * p, tmp, s);
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  if (cur != 0) {
    hipError_t e = hipMemcpyAsync(keys_a, keys_b, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals_a, vals_b, n * sizeof(int), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_ranges(int2* ranges, int n_keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_keys) ranges[i] = make_int2(0, 0);
}

__global__ __launch_bounds__(256) void k_finish(const uint32_t* keys, const int* vals, const int* entry_rec,
                                                int64_t n_max, const int* n_dev, int* sorted_rec, int2* ranges) {
  const int64_t n = items_of(n_dev, n_max);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int v = vals[i];
  sorted_rec[i] = entry_rec[v];
  uint32_t key = keys[i];
  if (i == 0 || keys[i - 1] != key) ranges[key].x = (int)i;
  if (i == n - 1 || keys[i + 1] != key) ranges[key].y = (int)(i + 1);
}

// Dispatch order of the tiles: heavy tiles (list longer than `split`) first,
// then the rest, each group longest first to a quantised length (one 8-bit
// radix pass; the sort is stable, so ties keep tile order). Heavy tiles start
// early instead of forming the tail of the launch, and consecutive blocks,
// which the hardware deals round-robin to the XCDs, spread them over all of
// them. Keys below 128 are exactly the heavy tiles.
__global__ __launch_bounds__(256) void k_tile_keys(const int2* ranges, int n_keys, int split, uint32_t* keys,
                                                   int* vals) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_keys) return;
  int2 r = ranges[i];
  int len = max(r.y - r.x, 0);
  uint32_t k;
  if (len > split)
    k = 127u - (uint32_t)min((len - split - 1) >> 5, 127);  // 32 entries a step
  else
    k = 255u - (uint32_t)min(len >> 2, 127);                 // 4 entries a step
  keys[i] = k;
  vals[i] = i;
}

// Block list of the render kernels from the ordered tiles: the first ns tiles
// (the heavy ones) get four blocks each, coded -(4 key + quadrant) - 1, then
// one block per remaining tile (its key), then blocks coded n_keys that exit
// at once (the grid is render_blocks()).
__global__ __launch_bounds__(256) void k_block_list(const uint32_t* sorted_keys, const int* order, int n_keys,
                                                   int* blocks) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = render_blocks(n_keys);
  if (t >= total) return;
  // ns = number of leading tiles with a key below 128
  int lo = 0, hi = n_keys;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (sorted_keys[mid] < 128u) lo = mid + 1; else hi = mid;
  }
  const int ns = lo;
  if (t < n_keys) {
    if (t < ns) {
#pragma unroll
      for (int q = 0; q < 4; ++q) blocks[4 * t + q] = -(4 * order[t] + q) - 1;
    } else {
      blocks[3 * ns + t] = order[t];
    }
  } else if (t >= n_keys + 3 * ns) {
    blocks[t] = n_keys;
  }
}

size_t order_tmp_ints(int n_keys) { return 4 * (size_t)n_keys + radix_tmp_ints(n_keys); }

hipError_t launch_tile_order(const int2* ranges, int n_keys, int split, int* blocks, int* tmp, hipStream_t s) {
  if (n_keys <= 0) return hipSuccess;
  uint32_t* ka = reinterpret_cast<uint32_t*>(tmp);
  uint32_t* kb = ka + n_keys;
  int* va = tmp + 2 * (size_t)n_keys;
  int* vb = tmp + 3 * (size_t)n_keys;
  int* rt = tmp + 4 * (size_t)n_keys;
  hipLaunchKernelGGL(k_tile_keys, dim3((n_keys + 255) / 256), dim3(256), 0, s, ranges, n_keys, split, ka, va);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = radix_pass(ka, va, kb, vb, n_keys, nullptr, 0, rt, s);
  if (e != hipSuccess) return e;
  int total = render_blocks(n_keys);
  hipLaunchKernelGGL(k_block_list, dim3((total + 255) / 256), dim3(256), 0, s, kb, vb, n_keys, blocks);
  return hipGetLastError();
}

hipError_t launch_finish_lists(const uint32_t* keys, const int* vals, const int* entry_rec, int64_t n,
                               const int* n_dev, int* sorted_rec, int2* ranges, int n_keys, bool ranges_cleared,
                               hipStream_t s) {
  if (!ranges_cleared)
    hipLaunchKernelGGL(k_fill_ranges, dim3((n_keys + 255) / 256), dim3(256), 0, s, ranges, n_keys);
  if (n > 0)
    hipLaunchKernelGGL(k_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, vals, entry_rec,
                       n, n_dev, sorted_rec, ranges);
  return hipGetLastError();
}

}  // namespace mb
