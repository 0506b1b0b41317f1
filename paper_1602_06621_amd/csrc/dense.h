// Dense and matrix-free paths of libmfe.
#pragma once

#include "common.h"

namespace mfe {

int dense_f64_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                          double* u_bar, double* v_bar);
int dense_f64_equilibrate_noalloc(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                                  double* u_bar, double* v_bar);
int dense_bf16_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                           double* u_bar, double* v_bar);
int operator_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                         double* u_bar, double* v_bar);
int dense_f64_lsqr(const mfe_matrix* A, const double* b, const double* d, const double* e, double tol,
                   int32_t max_iter, int32_t check_every, double* x, mfe_lsqr_info* info, hipStream_t s);
int dense_f64_residual(const mfe_matrix* A, const double* d, const double* e, double alpha, double beta,
                       double* rms, double* rms_nonempty, int64_t* n_empty, hipStream_t s);

}  // namespace mfe
