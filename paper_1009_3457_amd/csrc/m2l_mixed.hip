// Split-precision M2L contraction (BF16x3 / FP16x3 on MFMA).
#include "fmm2d_internal.h"
#include "m2l_mixed_bank.h"

namespace fmm2d {

bool m2l_mixed_supported(int p, int precision) {
  (void)p;
  (void)precision;
  return false;
}

size_t mixed_bank_bytes(int p, int precision) {
  (void)p;
  (void)precision;
  return 0;
}

int launch_mixed_ops(int p, int precision, void *ops, hipStream_t s) {
  (void)ops;
  (void)s;
  return set_error(FMM2D_EUNSUPPORTED_P, "precision %d is not built for p = %d", precision, p);
}

int launch_m2l_mixed(const float *M, const float *gb_in, float *L, float *b, int depth, int p, int lmin, int lmax,
                     bool adjoint, int precision, const void *ops, hipStream_t s) {
  (void)M; (void)gb_in; (void)L; (void)b; (void)depth; (void)lmin; (void)lmax; (void)adjoint; (void)ops; (void)s;
  return set_error(FMM2D_EUNSUPPORTED_P, "precision %d is not built for p = %d", precision, p);
}

}  // namespace fmm2d
