// Krylov vector kernels: deterministic dot products and the fused CG updates
// (the "vector inner product and other kernels" beside SpMV in CG and GMRES,
// Introduction).  All are HBM-bound streams.  Reductions are two-stage with a
// fixed order: grid-stride sum per thread -> wave butterfly -> 4 waves ->
// one partial per block; a one-block finish kernel then sums the partials in
// block order and updates the device-resident scalars.
#include "matrix.hpp"
#include "solvers.hpp"

namespace ck {

template <typename T>
int64_t dot_blocks(int64_t n) {
    int64_t g = ceil_div(n, 2048);
    if (g < 1)
        g = 1;
    return g < 1024 ? g : 1024;
}
template int64_t dot_blocks<double>(int64_t);
template int64_t dot_blocks<float>(int64_t);

}  // namespace ck

using ck::CgDev;

__device__ __forceinline__ bool skipped_v(const int *skip) { return skip != nullptr && *skip != 0; }

// partials[b] = sum over this block's grid-stride share of x_i * y_i
__global__ __launch_bounds__(256) void dot_partial(int64_t n, int64_t G,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   double *__restrict__ partials) {
    __shared__ double lds[4];
    const int64_t b = blockIdx.x;
    double s = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < n; i += G * 256)
        s += x[i] * y[i];
    s = ck::block_sum(s, lds);
    if (threadIdx.x == 0)
        partials[b] = s;
}

__global__ __launch_bounds__(256) void dot_finish(int64_t G, const double *__restrict__ partials,
                                                  double *__restrict__ out) {
    __shared__ double lds[4];
    const double t = ck::sum_partials(partials, G, lds);
    if (threadIdx.x == 0)
        out[0] = t;
}

// CG start from a residual already in r: p = r, partials of r.r
template <typename T>
__global__ __launch_bounds__(256) void cg_start(int64_t n, int64_t G, const T *__restrict__ r,
                                                T *__restrict__ p, T *__restrict__ partials,
                                                const CgDev<T> *cg) {
    __shared__ T lds[4];
    if (cg->state != ck::RUN)
        return;
    const int64_t b = blockIdx.x;
    T s = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < n; i += G * 256) {
        const T ri = r[i];
        p[i] = ri;
        s += ri * ri;
    }
    s = ck::block_sum(s, lds);
    if (threadIdx.x == 0)
        partials[b] = s;
}

// rho = r.r, relres = sqrt(rho)/bnorm; CONVERGED or BUDGET ends the run
template <typename T>
__global__ __launch_bounds__(256) void cg_start_finish(int64_t G, const T *__restrict__ partials,
                                                       CgDev<T> *cg) {
    __shared__ T lds[4];
    if (cg->state != ck::RUN)
        return;
    const T rho = ck::sum_partials(partials, G, lds);
    if (threadIdx.x == 0) {
        cg->rho = rho;
        cg->relres = sqrt((double)rho) / cg->bnorm;
        if (cg->relres <= cg->tol)
            cg->state = ck::CONVERGED;
        else if (cg->iter >= cg->max_iter)
            cg->state = ck::BUDGET;
    }
}

// partials of p.q, for configurations whose SpMV does not fuse the dot
template <typename T>
__global__ __launch_bounds__(256) void cg_sigma(int64_t n, int64_t G, const T *__restrict__ p,
                                                const T *__restrict__ q, T *__restrict__ partials,
                                                const CgDev<T> *cg) {
    __shared__ T lds[4];
    if (cg->state != ck::RUN)
        return;
    const int64_t b = blockIdx.x;
    T s = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < n; i += G * 256)
        s += p[i] * q[i];
    s = ck::block_sum(s, lds);
    if (threadIdx.x == 0)
        partials[b] = s;
}

// sigma = p.Ap; alpha = rho/sigma, or BREAKDOWN when sigma <= 0.  `go`
// tells the x/p update of this iteration whether to run.
template <typename T>
__global__ __launch_bounds__(256) void cg_sigma_finish(int64_t G, const T *__restrict__ partials,
                                                       CgDev<T> *cg) {
    __shared__ T lds[4];
    if (cg->state != ck::RUN) {
        if (threadIdx.x == 0)
            cg->go = 0;
        return;
    }
    const T sigma = ck::sum_partials(partials, G, lds);
    if (threadIdx.x == 0) {
        cg->sigma = sigma;
        cg->rho_prev = cg->rho;
        if (!(sigma > T(0))) {
            cg->state = ck::BREAKDOWN;
            cg->go = 0;
        } else {
            cg->alpha = cg->rho / sigma;
            cg->go = 1;
        }
    }
}

// r -= alpha q; partials of r.r (x is updated with p in cg_rho_update_xp,
// which reads p anyway)
template <typename T>
__global__ __launch_bounds__(256) void cg_update_r(int64_t n, int64_t G, T *__restrict__ r,
                                                   const T *__restrict__ q,
                                                   T *__restrict__ partials, const CgDev<T> *cg) {
    __shared__ T lds[4];
    if (cg->state != ck::RUN)
        return;
    const T alpha = cg->alpha;
    const int64_t b = blockIdx.x;
    T s = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < n; i += G * 256) {
        const T ri = r[i] - alpha * q[i];
        r[i] = ri;
        s += ri * ri;
    }
    s = ck::block_sum(s, lds);
    if (threadIdx.x == 0)
        partials[b] = s;
}

// The rho finish and the x and p updates in one kernel of G blocks (G = the
// number of r.r partials): every block sums the G partials itself, in the
// order a one-block finish would (same bits in every block), forms
// rho' = r.r, the convergence test on sqrt(rho')/bnorm and
// beta = rho'/rho_prev; it adds alpha p to its share of x and, unless
// converged, sets p = r + beta p there.  Block 0 alone stores the scalars.
// No block reads a field that block 0 stores: `go`, rho_prev and alpha were
// set by the sigma finish.
template <typename T>
__global__ __launch_bounds__(256) void cg_rho_update_xp(int64_t n, int64_t G,
                                                        const T *__restrict__ partials,
                                                        T *__restrict__ x, T *__restrict__ p,
                                                        const T *__restrict__ r, CgDev<T> *cg) {
    __shared__ T lds[4];
    __shared__ T beta_s;
    __shared__ int run_s;
    if (!cg->go)
        return;
    const T alpha = cg->alpha;
    const T rho_new = ck::sum_partials(partials, G, lds);
    if (threadIdx.x == 0) {
        const double relres = sqrt((double)rho_new) / cg->bnorm;
        const bool converged = relres <= cg->tol;
        const T beta = rho_new / cg->rho_prev;
        beta_s = beta;
        run_s = !converged;
        if (blockIdx.x == 0) {
            const int iter = cg->iter + 1;
            cg->beta = beta;
            cg->rho = rho_new;
            cg->iter = iter;
            cg->relres = relres;
            if (converged)
                cg->state = ck::CONVERGED;
            else if (iter >= cg->max_iter)
                cg->state = ck::BUDGET;
        }
    }
    __syncthreads();
    const T beta = beta_s;
    if (run_s) {
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += G * 256) {
            const T pi = p[i];
            x[i] += alpha * pi;
            p[i] = r[i] + beta * pi;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += G * 256)
            x[i] += alpha * p[i];
    }
}

// ---- small elementwise helpers -----------------------------------------------
template <typename D, typename S>
__global__ __launch_bounds__(256) void copy_cast(int64_t n, D *__restrict__ dst,
                                                 const S *__restrict__ src,
                                                 const int *__restrict__ skip) {
    if (skipped_v(skip))
        return;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        dst[i] = (D)src[i];
}

// dst = (D)(src * scale[0])  -- scale read from device memory
template <typename D>
__global__ __launch_bounds__(256) void scale_cast(int64_t n, D *__restrict__ dst,
                                                  const double *__restrict__ src,
                                                  const double *__restrict__ scale,
                                                  const int *__restrict__ skip) {
    if (skipped_v(skip))
        return;
    const double a = scale[0];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        dst[i] = (D)(src[i] * a);
}

// x += scale[0] * (double)d
template <typename S>
__global__ __launch_bounds__(256) void axpy_promote(int64_t n, double *__restrict__ x,
                                                    const S *__restrict__ d,
                                                    const double *__restrict__ scale,
                                                    const int *__restrict__ skip) {
    if (skipped_v(skip))
        return;
    const double a = scale[0];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        x[i] += a * (double)d[i];
}

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(int64_t n, T *__restrict__ dst, T v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        dst[i] = v;
}

// ---------------------------------------------------------------------------
namespace ck {

static int64_t stream_grid(int64_t n) {
    int64_t g = ceil_div(n, 256 * 4);
    if (g < 1)
        g = 1;
    return g < 8192 ? g : 8192;
}

ck_status launch_dot(int64_t n, const double *x, const double *y, double *partials, double *out,
                     hipStream_t s) {
    const int64_t G = dot_blocks<double>(n);
    hipLaunchKernelGGL(dot_partial, dim3(G), dim3(256), 0, s, n, G, x, y, partials);
    hipLaunchKernelGGL(dot_finish, dim3(1), dim3(256), 0, s, G, partials, out);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename T>
ck_status launch_cg_start(int64_t n, const T *r, T *p, T *partials, CgDev<T> *cg, hipStream_t s) {
    const int64_t G = dot_blocks<T>(n);
    hipLaunchKernelGGL((cg_start<T>), dim3(G), dim3(256), 0, s, n, G, r, p, partials, cg);
    hipLaunchKernelGGL((cg_start_finish<T>), dim3(1), dim3(256), 0, s, G, partials, cg);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename T>
ck_status launch_cg_sigma(int64_t n, const T *p, const T *q, T *partials, CgDev<T> *cg,
                          hipStream_t s) {
    const int64_t G = dot_blocks<T>(n);
    hipLaunchKernelGGL((cg_sigma<T>), dim3(G), dim3(256), 0, s, n, G, p, q, partials, cg);
    hipLaunchKernelGGL((cg_sigma_finish<T>), dim3(1), dim3(256), 0, s, G, partials, cg);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename T>
ck_status launch_cg_sigma_finish(int64_t G, T *partials, CgDev<T> *cg, hipStream_t s) {
    hipLaunchKernelGGL((cg_sigma_finish<T>), dim3(1), dim3(256), 0, s, G, partials, cg);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename T>
ck_status launch_cg_update(int64_t n, T *x, T *r, T *p, const T *q, T *partials, CgDev<T> *cg,
                           hipStream_t s) {
    const int64_t G = dot_blocks<T>(n);
    hipLaunchKernelGGL((cg_update_r<T>), dim3(G), dim3(256), 0, s, n, G, r, q, partials, cg);
    hipLaunchKernelGGL((cg_rho_update_xp<T>), dim3(G), dim3(256), 0, s, n, G, partials, x, p, r,
                       cg);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename D, typename S>
ck_status launch_copy(int64_t n, D *dst, const S *src, const int *skip, hipStream_t s) {
    hipLaunchKernelGGL((copy_cast<D, S>), dim3(stream_grid(n)), dim3(256), 0, s, n, dst, src,
                       skip);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename D>
ck_status launch_scale_cast(int64_t n, D *dst, const double *src, const double *scale,
                            const int *skip, hipStream_t s) {
    hipLaunchKernelGGL((scale_cast<D>), dim3(stream_grid(n)), dim3(256), 0, s, n, dst, src, scale,
                       skip);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename S>
ck_status launch_axpy_promote(int64_t n, double *x, const S *d, const double *scale,
                              const int *skip, hipStream_t s) {
    hipLaunchKernelGGL((axpy_promote<S>), dim3(stream_grid(n)), dim3(256), 0, s, n, x, d, scale,
                       skip);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename T>
ck_status launch_fill(int64_t n, T *dst, T v, hipStream_t s) {
    if (n <= 0)
        return CK_OK;
    hipLaunchKernelGGL((fill_kernel<T>), dim3(stream_grid(n)), dim3(256), 0, s, n, dst, v);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

#define CK_INST(T)                                                                          \
    template ck_status launch_cg_start<T>(int64_t, const T *, T *, T *, CgDev<T> *,         \
                                          hipStream_t);                                     \
    template ck_status launch_cg_sigma<T>(int64_t, const T *, const T *, T *, CgDev<T> *,   \
                                          hipStream_t);                                     \
    template ck_status launch_cg_sigma_finish<T>(int64_t, T *, CgDev<T> *, hipStream_t);    \
    template ck_status launch_cg_update<T>(int64_t, T *, T *, T *, const T *, T *,          \
                                           CgDev<T> *, hipStream_t);                        \
    template ck_status launch_scale_cast<T>(int64_t, T *, const double *, const double *,   \
                                            const int *, hipStream_t);                      \
    template ck_status launch_axpy_promote<T>(int64_t, double *, const T *, const double *, \
                                              const int *, hipStream_t);                    \
    template ck_status launch_fill<T>(int64_t, T *, T, hipStream_t);
CK_INST(double)
CK_INST(float)
template ck_status launch_fill<int>(int64_t, int *, int, hipStream_t);
template ck_status launch_fill<unsigned char>(int64_t, unsigned char *, unsigned char, hipStream_t);
template ck_status launch_copy<double, double>(int64_t, double *, const double *, const int *,
                                               hipStream_t);
template ck_status launch_copy<float, double>(int64_t, float *, const double *, const int *,
                                              hipStream_t);
template ck_status launch_copy<float, float>(int64_t, float *, const float *, const int *,
                                             hipStream_t);

}  // namespace ck
