// LSQR on the right-preconditioned operator A Rinv, with the recurrence state
// kept in device memory (launchers in lsqr.hip).
#pragma once
#include "sk_common.hpp"

namespace sk {

// Scalars of the Paige-Saunders recurrence. The stored left vector s relates
// to the current u by u = uscale * s; the next fused pass forms
// p = A (Rinv v) + coef * s.
struct LsqrDev {
  double alpha, beta, rhobar, phibar, anorm2, rnorm, arnorm, anorm, bnorm;
  double uscale, coef, tol, minus_one;
  int iters, done, converged, maxit;
};

// Number of workgroups (partial rows) of one fused pass over n rows.
int lsqr_pass_groups(int64_t n);
// p = A w + (*coefp) u (u <- p) and qv = [A^T p ; ||p||^2] (qv = part + groups*(m+1)).
// Skipped (both kernels return at once) while *donep != 0; donep may be null.
int launch_lsqr_pass(const double* A, int64_t lda, int64_t n, int m, const double* w, const double* coefp,
                     const int* donep, double* u, double* part, hipStream_t st);
// Writes tol, maxit and the constants read by the first pass (coef = -1).
int launch_lsqr_setup(LsqrDev* sd, double tol, int maxit, hipStream_t st);
// From qv of the pass p0 = A x0 - b: beta u1, alpha v1, w = v1, wv = Rinv v1.
// Rinv: R^{-1} (k x k row-major, upper); RinvT: its transpose. k <= 512.
int launch_lsqr_init(LsqrDev* sd, const double* qv, const double* Rinv, const double* RinvT, int k, double* v,
                     double* wd, double* y, double* wv, hipStream_t st);
// One iteration from qv of the pass p = A wv - alpha u (no-op once done).
int launch_lsqr_step(LsqrDev* sd, const double* qv, const double* Rinv, const double* RinvT, int k, double* v,
                     double* wd, double* y, double* wv, hipStream_t st);
// x = x0 + Rinv y
int launch_lsqr_finish(const double* Rinv, int k, const double* x0, const double* y, double* x, hipStream_t st);
// x = Rinv c
int launch_rinv_vec(const double* Rinv, int k, const double* c, double* x, hipStream_t st);

}  // namespace sk
