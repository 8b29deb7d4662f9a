// Cell-block helpers for the differentiable solve A(sigma) u = M s with
// A(sigma) = A_adv + sum_K sigma_K M_K, M_K a dense bs x bs cell block.
#include "airg.h"
#include "common.hpp"

using namespace airg;

namespace airg {
extern thread_local std::string g_last_error;
}

namespace {

// val[pos[K, a, b]] = base[pos[K, a, b]] + sigma_K M_K[a, b]
__global__ void k_bd_axpy(int64_t ncell, int bs, const double *__restrict__ mass, const double *__restrict__ sigma,
                          const int32_t *__restrict__ pos, const double *__restrict__ base,
                          double *__restrict__ val) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)bs * bs;
    if (t >= ncell * per) return;
    int64_t K = t / per;
    int32_t p = pos[t];
    val[p] = base[p] + sigma[K] * mass[t];
}

// y_K = M_K x_K
__global__ void k_bd_apply(int64_t ncell, int bs, const double *__restrict__ mass, const double *__restrict__ x,
                           double *__restrict__ y) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell * bs) return;
    int64_t K = t / bs;
    int a = (int)(t % bs);
    const double *m = mass + (K * bs + a) * bs;
    const double *xk = x + K * bs;
    double s = 0.0;
    for (int b = 0; b < bs; ++b) s += m[b] * xk[b];
    y[t] = s;
}

// out_K = scale * lam_K^T M_K u_K
__global__ void k_bd_bilinear(int64_t ncell, int bs, const double *__restrict__ mass, const double *__restrict__ u,
                              const double *__restrict__ lam, double scale, double *__restrict__ out) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= ncell) return;
    const double *m = mass + K * bs * bs;
    double s = 0.0;
    for (int a = 0; a < bs; ++a) {
        double r = 0.0;
        for (int b = 0; b < bs; ++b) r += m[a * bs + b] * u[K * bs + b];
        s += lam[K * bs + a] * r;
    }
    out[K] = scale * s;
}

template <class F>
airg_status guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return AIRG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return static_cast<airg_status>(e.status);
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return AIRG_ERR_HIP;
    }
}

}  // namespace

extern "C" {

airg_status airg_blockdiag_axpy(int64_t ncell, int32_t bs, const double *d_mass, const double *d_sigma,
                                const int32_t *d_pos, const double *d_base, double *d_val, void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(ncell >= 0 && bs >= 1 && bs <= 8 && d_mass && d_sigma && d_pos && d_base && d_val,
                     ST_INVALID_ARG, "bad argument");
        if (ncell == 0) return;
        int64_t work = ncell * bs * bs;
        k_bd_axpy<<<grid_for(work, 256), 256, 0, (hipStream_t)hip_stream>>>(ncell, bs, d_mass, d_sigma, d_pos, d_base,
                                                                           d_val);
        AIRG_LAUNCH_CHECK();
    });
}

airg_status airg_blockdiag_apply(int64_t ncell, int32_t bs, const double *d_mass, const double *d_x, double *d_y,
                                 void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(ncell >= 0 && bs >= 1 && bs <= 8 && d_mass && d_x && d_y, ST_INVALID_ARG, "bad argument");
        if (ncell == 0) return;
        k_bd_apply<<<grid_for(ncell * bs, 256), 256, 0, (hipStream_t)hip_stream>>>(ncell, bs, d_mass, d_x, d_y);
        AIRG_LAUNCH_CHECK();
    });
}

airg_status airg_blockdiag_bilinear(int64_t ncell, int32_t bs, const double *d_mass, const double *d_u,
                                    const double *d_lam, double scale, double *d_out, void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(ncell >= 0 && bs >= 1 && bs <= 8 && d_mass && d_u && d_lam && d_out, ST_INVALID_ARG,
                     "bad argument");
        if (ncell == 0) return;
        k_bd_bilinear<<<grid_for(ncell, 256), 256, 0, (hipStream_t)hip_stream>>>(ncell, bs, d_mass, d_u, d_lam, scale,
                                                                                d_out);
        AIRG_LAUNCH_CHECK();
    });
}

}  // extern "C"
