// Internal declarations shared by the HIP translation units of libfmm2d.so.
// Nothing here is part of the public ABI (include/fmm2d.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "fmm2d.h"

namespace fmm2d {

constexpr int kMaxDepth = 12;

// ------------------------------------------------------------ box indexing --
// Level l occupies [level_off(l), level_off(l+1)) in every per-box array; inside a
// level boxes are in Morton order (bit 2b of the index = bit b of ix).

__host__ __device__ inline int64_t level_off(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }

// Spread the low 16 bits of v to the even bit positions.
__host__ __device__ inline uint32_t spread2(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// Inverse of spread2: gather the even bits of v.
__host__ __device__ inline uint32_t compact2(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0f0f0f0fu;
  v = (v | (v >> 4)) & 0x00ff00ffu;
  v = (v | (v >> 8)) & 0x0000ffffu;
  return v;
}

__host__ __device__ inline uint32_t morton2(uint32_t ix, uint32_t iy) {
  return spread2(ix) | (spread2(iy) << 1);
}

__host__ __device__ inline void unmorton2(uint32_t m, uint32_t &ix, uint32_t &iy) {
  ix = compact2(m);
  iy = compact2(m >> 1);
}

// ------------------------------------------------------------ small math --

struct cd {  // complex double
  double re, im;
};

__host__ __device__ inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Number of supported orders and their index (p = 8, 12, 16, 20).
__host__ __device__ inline bool p_supported(int p) { return p == 8 || p == 12 || p == 16 || p == 20; }

// ------------------------------------------------------------ errors --------

int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
int check_launch(const char *what);  // FMM2D_OK or FMM2D_EHIP after a kernel launch

// ------------------------------------------------------------ launchers -----
// Each launcher assumes validated arguments and only enqueues work.

// Workspace of the tree build's radix sort for n points: keys and values,
// both double-buffered, the per-chunk digit counts and the scan's block totals.
namespace tree_ws {
constexpr int kChunk = 1024;      // items per sort chunk
constexpr int kDigits = 16;       // values of one 4-bit digit
constexpr int kScanBlock = 4096;  // values per scan block
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr int64_t nchunks(int64_t n) { return (n + kChunk - 1) / kChunk; }
constexpr int64_t scan_blocks(int64_t m) { return (m + kScanBlock - 1) / kScanBlock; }
constexpr size_t bytes(int64_t n) {
  return 4 * align256(size_t(n) * 4) + align256(size_t(kDigits) * size_t(nchunks(n)) * 4) +
         align256(size_t(scan_blocks(int64_t(kDigits) * nchunks(n))) * 4);
}
}  // namespace tree_ws

int launch_build_tree(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                      uint32_t *domain_flag, void *ws, hipStream_t s);
size_t build_tree_ws_bytes(int64_t n, int depth);
// The same with the workspace in the library's own device array (n at most
// kNoAllocMaxPoints); looks the array up on the current device first.
constexpr int64_t kNoAllocMaxPoints = int64_t(1) << 22;
int launch_build_tree_noalloc(const float *xy, int64_t n, int depth, int32_t *perm, int32_t *leaf_start,
                              uint32_t *domain_flag, hipStream_t s);
int launch_gather(const float *src, const int32_t *perm, int64_t n, int width, float *dst, bool scatter,
                  hipStream_t s);

int launch_p2m(const float *xy, const float *q, const int32_t *ls, int depth, int p, float *M, hipStream_t s);
int launch_m2m(float *M, int depth, int p, hipStream_t s);
int launch_l2l(const float *Lm2l, const float *bm2l, double *L, double *b, int depth, int p, hipStream_t s);
int launch_l2p(const float *txy, const int32_t *tls, int64_t nt, const double *L, const double *b, int depth,
               int p, float *phi, float *field, hipStream_t s);
int launch_p2p(const float *xy, const float *q, const int32_t *ls, const float *txy, const int32_t *tls,
               int64_t nt, int depth, float *phi, float *field, hipStream_t s);

int launch_l2p_backward(const float *txy, const int32_t *tls, const float *cphi, const float *cfield,
                        int depth, int p, double *gL, double *gb, hipStream_t s);
int launch_l2l_backward(double *gL, double *gb, float *gLm2l, float *gbm2l, int depth, int p, hipStream_t s);
int launch_m2m_backward(float *gM, int depth, int p, hipStream_t s);
int launch_p2m_backward(const float *xy, const float *q, const int32_t *ls, int64_t n, int depth, int p,
                        const float *gM, float *gq, float *G, hipStream_t s);
int launch_p2p_backward(const float *xy, const float *q, const int32_t *ls, int64_t n, const float *txy,
                        const int32_t *tls, int depth, const float *cphi, const float *cfield, float *gq,
                        float *G, hipStream_t s);

// M2L operator banks and contraction kernels.
size_t m2l_ops_bytes(int p, int precision);
int launch_m2l_ops(int p, int precision, void *ops, hipStream_t s);
int launch_m2l_f32(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                   bool adjoint, const void *ops, hipStream_t s);
int launch_m2l_pascal(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                      bool adjoint, const void *ops, hipStream_t s);
bool m2l_mixed_supported(int p, int precision);
int num_cus();  // compute units of the current device
// b(t) for every box of levels lmin..lmax from the forward log rows r[slot][k]
// (complex FP32, slot = (ox+3) + 7 (oy+3)); used when the MFMA tiles have no
// spare rows for it
int launch_m2l_logrow_fwd(const float *M, float *b, int p, int lmin, int lmax, const float *r, hipStream_t s);
// its transpose, added into gM for every source box of levels lmin..lmax
int launch_m2l_logrow_bwd(const float *gb, float *gM, int p, int lmin, int lmax, const float *r, hipStream_t s);
// the Hankel form (FP64 frequency-domain accumulation), with the log row's pass
int launch_m2l_hankel(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                      bool adjoint, const void *ops, hipStream_t s);
int launch_m2l_mixed(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin,
                     int lmax, bool adjoint, int precision, const void *ops, hipStream_t s);

}  // namespace fmm2d
