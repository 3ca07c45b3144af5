// Initialization stage (Sec. 2.1, stage 1): leaf assignment and a stable sort
// of the points by leaf Morton key, plus gather/scatter of per-point rows.
//
// The sort is a least-significant-digit radix sort over 4-bit digits of the
// 2*depth-bit key.  Each pass is: per-chunk digit counts, an exclusive scan
// over (digit, chunk) (three short kernels), and a scatter in which every
// item's rank among equal digits of its chunk comes from wave ballots, so
// each pass is stable and the whole result is deterministic.
#include "fmm2d_internal.h"

namespace fmm2d {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 4;
constexpr int kChunk = kSortThreads * kSortRounds;  // items per chunk
constexpr int kDigits = 16;
static_assert(kChunk == tree_ws::kChunk && kDigits == tree_ws::kDigits, "workspace layout");

using tree_ws::align256;
constexpr int64_t nchunks_of(int64_t n) { return tree_ws::nchunks(n); }

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;                         // values per thread
constexpr int kScanBlock = kScanThreads * kScanPer;  // 4096 values per block
static_assert(kScanBlock == tree_ws::kScanBlock, "workspace layout");

constexpr int64_t scan_blocks(int64_t m) { return tree_ws::scan_blocks(m); }

struct TreeWs {
  uint32_t *keys[2];
  int32_t *vals[2];
  uint32_t *count;  // [kDigits][nchunks]
  uint32_t *part;   // [scan_blocks(kDigits * nchunks)]
};

static TreeWs carve(void *ws, int64_t n) {
  char *p = static_cast<char *>(ws);
  TreeWs w;
  const size_t kb = align256(size_t(n) * 4);
  w.keys[0] = reinterpret_cast<uint32_t *>(p); p += kb;
  w.keys[1] = reinterpret_cast<uint32_t *>(p); p += kb;
  w.vals[0] = reinterpret_cast<int32_t *>(p); p += kb;
  w.vals[1] = reinterpret_cast<int32_t *>(p); p += kb;
  w.count = reinterpret_cast<uint32_t *>(p); p += align256(size_t(kDigits) * nchunks_of(n) * 4);
  w.part = reinterpret_cast<uint32_t *>(p);
  return w;
}

size_t build_tree_ws_bytes(int64_t n, int depth) {
  (void)depth;
  return tree_ws::bytes(n);
}

// The domain flag starts at zero on the stream (a kernel, not a memset, so
// the call can also be recorded into a graph).
__global__ void clear_flag_kernel(uint32_t *__restrict__ flag) { *flag = 0u; }

// Leaf key of every point; flags points outside [0,1]^2 (NaN included).
__global__ void leaf_keys_kernel(const float2 *__restrict__ xy, int64_t n, int depth, uint32_t *__restrict__ keys,
                                 int32_t *__restrict__ vals, uint32_t *__restrict__ flag) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const float2 p = xy[i];
  const bool inside = (p.x >= 0.f && p.x <= 1.f && p.y >= 0.f && p.y <= 1.f);
  if (!inside) atomicOr(flag, 1u);
  const float side = float(1 << depth);  // x * 2^depth is exact in FP32
  const int lim = (1 << depth) - 1;
  int ix = inside ? min(int(floorf(p.x * side)), lim) : 0;
  int iy = inside ? min(int(floorf(p.y * side)), lim) : 0;
  keys[i] = morton2(uint32_t(ix), uint32_t(iy));
  vals[i] = int32_t(i);
}

__global__ __launch_bounds__(kSortThreads) void digit_count_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                                   int shift, int64_t nchunks,
                                                                   uint32_t *__restrict__ count) {
  __shared__ uint32_t hist[kDigits];
  if (threadIdx.x < kDigits) hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * int64_t(kChunk);
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&hist[(keys[i] >> shift) & (kDigits - 1)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kDigits) count[threadIdx.x * nchunks + blockIdx.x] = hist[threadIdx.x];
}

// In-place exclusive scan of m values (the (digit, chunk) counts), in three
// coalesced passes: per-block totals of 4096 values, a scan of those totals by
// one workgroup, and a per-block scan that adds its block's offset.

__device__ inline void load16(const uint32_t *__restrict__ a, int64_t m, int64_t i0, uint32_t (&v)[kScanPer]) {
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) v[e] = (i0 + e < m) ? a[i0 + e] : 0u;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t *__restrict__ a, int64_t m,
                                                                   uint32_t *__restrict__ part) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  uint32_t v[kScanPer];
  load16(a, m, blockIdx.x * int64_t(kScanBlock) + threadIdx.x * int64_t(kScanPer), v);
  uint32_t s = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) s += v[e];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) t += wsum[w];
    part[blockIdx.x] = t;
  }
}

// exclusive scan of the nb block totals by one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void scan_partials_kernel(uint32_t *__restrict__ part, int64_t nb) {
  __shared__ uint32_t buf[1024];
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? part[i] : 0u;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {  // Hillis-Steele inclusive scan
      const uint32_t u = (int(threadIdx.x) >= d) ? buf[threadIdx.x - d] : 0u;
      __syncthreads();
      buf[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < nb) part[i] = carry + buf[threadIdx.x] - v;
    carry += buf[1023];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(uint32_t *__restrict__ a, int64_t m,
                                                                  const uint32_t *__restrict__ part) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int64_t i0 = blockIdx.x * int64_t(kScanBlock) + threadIdx.x * int64_t(kScanPer);
  uint32_t v[kScanPer];
  load16(a, m, i0, v);
  uint32_t s = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) s += v[e];
  // exclusive scan of the thread sums within the wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t off = part[blockIdx.x] + inc - s;
  for (int w = 0; w < wave; ++w) off += wsum[w];
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    if (i0 + e < m) a[i0 + e] = off;
    off += v[e];
  }
}

__global__ __launch_bounds__(kSortThreads) void digit_scatter_kernel(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    int32_t *__restrict__ vout, int64_t n, int shift, int64_t nchunks, const uint32_t *__restrict__ offset) {
  __shared__ uint32_t running[kDigits];
  __shared__ uint32_t wave_cnt[kSortThreads / 64][kDigits];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x < kDigits) running[threadIdx.x] = offset[threadIdx.x * nchunks + blockIdx.x];
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = blockIdx.x * int64_t(kChunk);
  for (int r = 0; r < kSortRounds; ++r) {
    __syncthreads();
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    const bool live = i < n;
    const uint32_t key = live ? kin[i] : 0u;
    const int dig = live ? int((key >> shift) & (kDigits - 1)) : -1;
    int rank = 0;
    for (int v = 0; v < kDigits; ++v) {
      const uint64_t m = __ballot(dig == v);
      if (dig == v) rank = __popcll(m & lt_mask);
      if (lane == 0) wave_cnt[wave][v] = uint32_t(__popcll(m));
    }
    __syncthreads();
    if (live) {
      uint32_t pos = running[dig] + uint32_t(rank);
      for (int w = 0; w < wave; ++w) pos += wave_cnt[w][dig];
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();
    if (threadIdx.x < kDigits) {
      uint32_t add = 0;
      for (int w = 0; w < kSortThreads / 64; ++w) add += wave_cnt[w][threadIdx.x];
      running[threadIdx.x] += add;
    }
  }
}

// leaf_start[m] = first sorted position whose key is >= m (binary search).
__global__ void leaf_start_kernel(const uint32_t *__restrict__ keys, int64_t n, int64_t nleaf,
                                  int32_t *__restrict__ leaf_start) {
  const int64_t m = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (m > nleaf) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(keys[mid]) < m) lo = mid + 1;
    else hi = mid;
  }
  leaf_start[m] = int32_t(lo);
}

__global__ void copy_i32_kernel(const int32_t *__restrict__ a, int32_t *__restrict__ b, int64_t n) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) b[i] = a[i];
}

int launch_build_tree(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                      uint32_t *domain_flag, void *ws, hipStream_t s) {
  TreeWs w = carve(ws, n);
  const int64_t nleaf = int64_t(1) << (2 * depth);
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, domain_flag);
  int cur = 0;
  if (n > 0) {
    const int64_t nchunks = nchunks_of(n);
    const unsigned gblocks = unsigned((n + 255) / 256);
    hipLaunchKernelGGL(leaf_keys_kernel, dim3(gblocks), dim3(256), 0, s, reinterpret_cast<const float2 *>(xy), n,
                       depth, w.keys[0], w.vals[0], domain_flag);
    const int bits = 2 * depth;
    for (int shift = 0; shift < bits; shift += 4) {
      hipLaunchKernelGGL(digit_count_kernel, dim3(unsigned(nchunks)), dim3(kSortThreads), 0, s, w.keys[cur], n,
                         shift, nchunks, w.count);
      const int64_t m = int64_t(kDigits) * nchunks, nb = scan_blocks(m);
      hipLaunchKernelGGL(scan_reduce_kernel, dim3(unsigned(nb)), dim3(kScanThreads), 0, s, w.count, m, w.part);
      hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, s, w.part, nb);
      hipLaunchKernelGGL(scan_apply_kernel, dim3(unsigned(nb)), dim3(kScanThreads), 0, s, w.count, m, w.part);
      hipLaunchKernelGGL(digit_scatter_kernel, dim3(unsigned(nchunks)), dim3(kSortThreads), 0, s, w.keys[cur],
                         w.vals[cur], w.keys[cur ^ 1], w.vals[cur ^ 1], n, shift, nchunks, w.count);
      cur ^= 1;
    }
    hipLaunchKernelGGL(copy_i32_kernel, dim3(gblocks), dim3(256), 0, s, w.vals[cur], perm, n);
  }
  hipLaunchKernelGGL(leaf_start_kernel, dim3(unsigned((nleaf + 1 + 255) / 256)), dim3(256), 0, s, w.keys[cur], n,
                     nleaf, leaf_start);
  return check_launch("build_tree");
}

__global__ void gather_kernel(const float *__restrict__ src, const int32_t *__restrict__ perm, int64_t n, int width,
                              float *__restrict__ dst, bool scatter) {
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= n * width) return;
  const int64_t i = e / width;
  const int c = int(e - i * width);
  if (scatter) dst[int64_t(perm[i]) * width + c] = src[e];
  else dst[e] = src[int64_t(perm[i]) * width + c];
}

// Rows of 1, 2 or 4 floats (charges, positions, complex values; pairs of
// complex values) move as one vector access per row: no index division, and
// one load of perm per row.
template <typename V>
__global__ void gather_rows_kernel(const V *__restrict__ src, const int32_t *__restrict__ perm, int64_t n,
                                   V *__restrict__ dst, bool scatter) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  if (scatter) dst[j] = src[i];
  else dst[i] = src[j];
}

template <typename V>
void launch_rows(const float *src, const int32_t *perm, int64_t n, float *dst, bool scatter, hipStream_t s) {
  hipLaunchKernelGGL(gather_rows_kernel<V>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const V *>(src), perm, n, reinterpret_cast<V *>(dst), scatter);
}

int launch_gather(const float *src, const int32_t *perm, int64_t n, int width, float *dst, bool scatter,
                  hipStream_t s) {
  if (n == 0) return FMM2D_OK;
  const uintptr_t align = reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst);
  if (width == 1) launch_rows<float>(src, perm, n, dst, scatter, s);
  else if (width == 2 && align % 8 == 0) launch_rows<float2>(src, perm, n, dst, scatter, s);
  else if (width == 4 && align % 16 == 0) launch_rows<float4>(src, perm, n, dst, scatter, s);
  else {
    const int64_t tot = n * width;
    hipLaunchKernelGGL(gather_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, src, perm, n, width, dst,
                       scatter);
  }
  return check_launch(scatter ? "scatter" : "gather");
}

}  // namespace fmm2d
