// extern "C" entry points of airg_steps.h: each setup step on device buffers.
#include <cmath>
#include <cstring>
#include <string>

#include "airg_steps.h"
#include "cfsplit.hpp"
#include "csr.hpp"
#include "hierarchy.hpp"
#include "spgemm.hpp"
#include "transfer.hpp"

using namespace airg;

struct airg_csr {
    Csr m;
};

namespace airg {
extern thread_local std::string g_last_error;
}

namespace {

template <class F>
airg_status guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return AIRG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return static_cast<airg_status>(e.status);
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return AIRG_ERR_OOM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return AIRG_ERR_HIP;
    } catch (...) {
        g_last_error = "unknown error";
        return AIRG_ERR_HIP;
    }
}

CsrView mk(int64_t nr, int64_t nc, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v) {
    AIRG_REQUIRE(nr >= 0 && nc >= 0 && nnz >= 0 && nr < ((int64_t)1 << 31) && nc < ((int64_t)1 << 31) &&
                     nnz < ((int64_t)1 << 31),
                 ST_INVALID_ARG, "size out of range");
    AIRG_REQUIRE(rp && (nnz == 0 || (ci && v)), ST_INVALID_ARG, "null matrix pointer");
    return CsrView{(int32_t)nr, (int32_t)nc, nnz, rp, ci, v, nullptr};
}

airg_csr *wrap(Csr &&m) {
    auto *o = new airg_csr;
    o->m = std::move(m);
    return o;
}

}  // namespace

extern "C" {

airg_status airg_csr_info(const airg_csr *A, int64_t *nrows, int64_t *ncols, int64_t *nnz) {
    return guarded([&] {
        AIRG_REQUIRE(A, ST_INVALID_ARG, "null matrix");
        if (nrows) *nrows = A->m.nr;
        if (ncols) *ncols = A->m.nc;
        if (nnz) *nnz = A->m.nnz;
    });
}

airg_status airg_csr_to_host(const airg_csr *A, int32_t *h_rowptr, int32_t *h_col, double *h_val) {
    return guarded([&] {
        AIRG_REQUIRE(A, ST_INVALID_ARG, "null matrix");
        hipStream_t s = A->m.rp.s;
        if (h_rowptr) d2h(h_rowptr, A->m.rp.p, (size_t)A->m.nr + 1, s);
        if (h_col) d2h(h_col, A->m.ci.p, (size_t)A->m.nnz, s);
        if (h_val) d2h(h_val, A->m.v.p, (size_t)A->m.nnz, s);
    });
}

void airg_csr_free(airg_csr *A) { delete A; }

airg_status airg_strength(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                          const double *d_val, double alpha, uint8_t *d_strong, int32_t *d_deg, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_strong, ST_INVALID_ARG, "null output");
        StrengthGraph G = strength_graph(A, alpha, s);
        d2d(d_strong, G.strong.p, (size_t)nnz, s);
        if (d_deg) strength_degree(G, d_deg, s);
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_pmisr(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col, const double *d_val,
                       double alpha, const uint32_t *d_h, uint64_t seed, int32_t level, int32_t max_rounds,
                       int8_t *d_cf, int32_t *rounds, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_cf && max_rounds >= 0, ST_INVALID_ARG, "bad argument");
        StrengthGraph G = strength_graph(A, alpha, s);
        int r = pmisr(A, G, d_h, max_rounds, d_cf, s, seed, level);
        if (rounds) *rounds = r;
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_ddc(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col, const double *d_val,
                     double alpha_diag, const int8_t *d_cf_in, int8_t *d_cf_out, double *d_theta,
                     void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_cf_in && d_cf_out, ST_INVALID_ARG, "null marker array");
        ddc(A, alpha_diag, d_cf_in, d_cf_out, d_theta, s);
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_ddc_fraction_threshold(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                                        const double *d_val, const int8_t *d_cf, double fraction,
                                        double *alpha_diag, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_cf && alpha_diag, ST_INVALID_ARG, "null argument");
        *alpha_diag = ddc_fraction_threshold(A, d_cf, fraction, s);
    });
}

airg_status airg_ddc_fraction_threshold_noalloc(int64_t n, int64_t nnz, const int32_t *d_rowptr,
                                                const int32_t *d_col, const double *d_val, const int8_t *d_cf,
                                                double fraction, double *alpha_diag, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_cf && alpha_diag, ST_INVALID_ARG, "null argument");
        *alpha_diag = ddc_fraction_threshold_noalloc(A, d_cf, fraction, s);
    });
}

int64_t airg_ddc_fraction_threshold_noalloc_max_rows(void) { return ddc_fraction_noalloc_max_rows(); }

airg_status airg_cf_split(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                          const double *d_val, const airg_opts *opts, int32_t level, int8_t *d_cf, int64_t *n_f,
                          int64_t *n_c, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(opts && d_cf, ST_INVALID_ARG, "null argument");
        CfParams p{opts->strong_threshold, opts->ddc_threshold, opts->ddc_fraction, opts->pmisr_max_rounds,
                   opts->seed};
        auto [nF, nC] = cf_split(A, p, level, d_cf, s);
        if (n_f) *n_f = nF;
        if (n_c) *n_c = nC;
    });
}

airg_status airg_extract(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                         const double *d_val, const int8_t *d_cf, int8_t rowsel, int8_t colsel, airg_csr **out,
                         void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_cf && out && (rowsel == CF_F || rowsel == CF_C) && (colsel == CF_F || colsel == CF_C),
                     ST_INVALID_ARG, "bad argument");
        *out = nullptr;
        DBuf<int32_t> rank((size_t)n, s);
        auto [nF, nC] = cf_ranks(d_cf, (int32_t)n, rank.p, s);
        int32_t nr = rowsel == CF_F ? nF : nC, nc = colsel == CF_F ? nF : nC;
        *out = wrap(extract_block(A, d_cf, rank.p, rowsel, colsel, nr, nc, s));
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_spmv(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                      const double *d_val, const double *d_x, double *d_y, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(nrows, ncols, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_x && d_y, ST_INVALID_ARG, "null vector");
        spmv(A, d_x, d_y, nullptr, SPMV_SET, s);
    });
}

airg_status airg_gauss_rhs(int64_t n, uint64_t seed, int32_t level, double *d_b, void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(d_b && n >= 0, ST_INVALID_ARG, "bad argument");
        gauss_rhs(n, seed, level, d_b, (hipStream_t)hip_stream);
    });
}

airg_status airg_tsqr_r(int64_t rows, int32_t cols, const double *d_K, double *h_R, double *h_colnorm,
                        void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(d_K && h_R && h_colnorm && rows > 0, ST_INVALID_ARG, "bad argument");
        tsqr_r(d_K, rows, cols, h_R, h_colnorm, (hipStream_t)hip_stream);
    });
}

airg_status airg_gmres_poly(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                            const double *d_val, uint64_t seed, int32_t level, int32_t m, double *h_alpha,
                            double *h_R, double *h_colnorm, int32_t *used, void *hip_stream) {
    return guarded([&] {
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(h_alpha, ST_INVALID_ARG, "null output");
        PolyInfo P = gmres_poly(A, seed, level, m, (hipStream_t)hip_stream);
        for (int k = 0; k < m; ++k) h_alpha[k] = P.alpha[k];
        if (h_R) std::memcpy(h_R, P.R, sizeof(double) * (m + 1) * (m + 1));
        if (h_colnorm) std::memcpy(h_colnorm, P.colnorm, sizeof(double) * (m + 1));
        if (used) *used = P.used;
    });
}

airg_status airg_poly_fixed_sparsity(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                                     const double *d_val, int32_t nalpha, const double *h_alpha, double *d_out_val,
                                     void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(h_alpha && d_out_val, ST_INVALID_ARG, "null argument");
        poly_fixed_sparsity(A, h_alpha, nalpha, d_out_val, s);
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_spgemm(int64_t m, int64_t k, int64_t nnz_a, const int32_t *d_arp, const int32_t *d_acol,
                        const double *d_aval, int64_t ncols_b, int64_t nnz_b, const int32_t *d_brp,
                        const int32_t *d_bcol, const double *d_bval, airg_csr **out, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(m, k, nnz_a, d_arp, d_acol, d_aval);
        CsrView B = mk(k, ncols_b, nnz_b, d_brp, d_bcol, d_bval);
        AIRG_REQUIRE(out, ST_INVALID_ARG, "null output");
        *out = nullptr;
        *out = wrap(spgemm(A, B, s));
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_drop(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                      const double *d_val, double tau, int32_t keep_diag, int32_t negate, airg_csr **out,
                      void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(nrows, ncols, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(out, ST_INVALID_ARG, "null output");
        *out = nullptr;
        *out = wrap(drop_rows(A, tau, keep_diag != 0, negate != 0, s));
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_onepoint_w(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                            const double *d_val, const int8_t *d_cf, int32_t weight_mode, airg_csr **out,
                            void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(d_cf && out, ST_INVALID_ARG, "null argument");
        *out = nullptr;
        DBuf<int32_t> rank((size_t)n, s);
        auto [nF, nC] = cf_ranks(d_cf, (int32_t)n, rank.p, s);
        Csr P, W;
        onepoint_prolongator(A, d_cf, rank.p, nF, nC, weight_mode, &P, &W, s);
        *out = wrap(std::move(W));
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_transpose(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *d_rowptr,
                           const int32_t *d_col, const double *d_val, airg_csr **out, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(nrows, ncols, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(out, ST_INVALID_ARG, "null output");
        *out = nullptr;
        *out = wrap(transpose(A, s));
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_level_build(int64_t n, int64_t nnz, const int32_t *d_rowptr, const int32_t *d_col,
                             const double *d_val, const airg_opts *opts, int32_t level, const double *h_alpha_in,
                             int8_t *d_cf, double *h_alpha_out, airg_csr **ainv, airg_csr **z, airg_csr **w,
                             airg_csr **ac, void *hip_stream) {
    return guarded([&] {
        hipStream_t s = (hipStream_t)hip_stream;
        CsrView A = mk(n, n, nnz, d_rowptr, d_col, d_val);
        AIRG_REQUIRE(opts, ST_INVALID_ARG, "null opts");
        AIRG_REQUIRE(opts->poly_order >= 0 && opts->poly_order + 2 <= kMaxPolyCols, ST_INVALID_ARG,
                     "poly_order out of range");
        LevelOut L = build_one_level(A, *opts, opts->seed, level, h_alpha_in, s);
        if (d_cf) d2d(d_cf, L.cf.p, (size_t)n, s);
        if (h_alpha_out)
            for (int k = 0; k <= opts->poly_order; ++k) h_alpha_out[k] = L.poly.alpha[k];
        if (ainv) *ainv = wrap(std::move(L.Ainv));
        if (z) *z = wrap(std::move(L.Z));
        if (w) *w = wrap(std::move(L.W));
        if (ac) *ac = wrap(std::move(L.Ac));
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

}  // extern "C"
