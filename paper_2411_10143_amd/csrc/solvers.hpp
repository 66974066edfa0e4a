// Internal launch interface of the Krylov kernels (vecops.hip, gmres.hip) and
// the host drivers (solvers.cpp).
#pragma once

#include "matrix.hpp"

namespace ck {

ck_status launch_dot(int64_t n, const double *x, const double *y, double *partials,
                     double *out, hipStream_t s);
template <typename T>
ck_status launch_cg_start(int64_t n, const T *r, T *p, T *partials, CgDev<T> *cg, hipStream_t s);
template <typename T>
ck_status launch_cg_sigma(int64_t n, const T *p, const T *q, T *partials, CgDev<T> *cg,
                          hipStream_t s);
// finishes sigma/alpha from the G partials a fused SpMV launch wrote
template <typename T>
ck_status launch_cg_sigma_finish(int64_t G, T *partials, CgDev<T> *cg, hipStream_t s);
template <typename T>
ck_status launch_cg_update(int64_t n, T *x, T *r, T *p, const T *q, T *partials, CgDev<T> *cg,
                           hipStream_t s);
template <typename D, typename S>
ck_status launch_copy(int64_t n, D *dst, const S *src, const int *skip, hipStream_t s);
template <typename D>
ck_status launch_scale_cast(int64_t n, D *dst, const double *src, const double *scale,
                            const int *skip, hipStream_t s);
template <typename S>
ck_status launch_axpy_promote(int64_t n, double *x, const S *d, const double *scale,
                              const int *skip, hipStream_t s);
template <typename T>
ck_status launch_fill(int64_t n, T *dst, T v, hipStream_t s);

// GMRES(m) pieces; V holds m+1 basis columns of length ldv.
int64_t gm_blocks(int64_t n);
template <typename T>
ck_status launch_gm_cycle_start(int64_t n, const double *r64, T *v0, double *partials64,
                                GmDev<T> *st, hipStream_t s);
template <typename T>
ck_status launch_gm_arnoldi(int64_t n, int j, T *V, int64_t ldv, T *partials, GmDev<T> *st,
                            hipStream_t s);
template <typename T>
ck_status launch_gm_cycle_end(int64_t n, double *x, const T *V, int64_t ldv, GmDev<T> *st,
                              hipStream_t s);

}  // namespace ck
