// Entry points not built yet report MFE_EUNSUPPORTED.
#include "dense.h"
#include "sparse.h"

namespace mfe {
int dense_f64_equilibrate(const mfe_matrix*, const mfe_equil_params*, double*, double*, double*, double*) {
  return set_error(MFE_EUNSUPPORTED, "dense FP64 path not built");
}
int dense_bf16_equilibrate(const mfe_matrix*, const mfe_equil_params*, double*, double*, double*, double*) {
  return set_error(MFE_EUNSUPPORTED, "dense BF16 path not built");
}
int operator_equilibrate(const mfe_matrix*, const mfe_equil_params*, double*, double*, double*, double*) {
  return set_error(MFE_EUNSUPPORTED, "operator path not built");
}
int dense_f64_lsqr(const mfe_matrix*, const double*, const double*, const double*, double, int32_t, int32_t,
                   double*, mfe_lsqr_info*, hipStream_t) {
  return set_error(MFE_EUNSUPPORTED, "dense LSQR not built");
}
int dense_f64_residual(const mfe_matrix*, const double*, const double*, double, double, double*, double*,
                       int64_t*, hipStream_t) {
  return set_error(MFE_EUNSUPPORTED, "dense residual not built");
}
int plan_lsqr(mfe_plan*, const double*, const double*, const double*, double, int32_t, int32_t, double*,
              mfe_lsqr_info*, hipStream_t) {
  return set_error(MFE_EUNSUPPORTED, "sparse LSQR not built");
}
int plan_residual(mfe_plan*, const double*, const double*, double, double, double*, double*, int64_t*,
                  hipStream_t) {
  return set_error(MFE_EUNSUPPORTED, "sparse residual not built");
}
}  // namespace mfe
