// extern "C" entry points of airg.h: status/error layer, handle, setup over
// one or many independent segments, forward and adjoint solves, inspection.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "airg.h"
#include "batch.hpp"
#include "csr.hpp"
#include "hierarchy.hpp"
#include "segmented.hpp"

using namespace airg;

struct airg_handle {
    airg_opts opt{};
    int64_t n = 0;
    std::vector<int64_t> seg;                 // nseg + 1 row offsets
    std::vector<uint64_t> seeds;
    std::vector<std::unique_ptr<Hier>> fwd;   // one hierarchy per segment (single and sequential forms)
    std::unique_ptr<SegHier> segh;            // all segments in one batch hierarchy (batched form)
    std::vector<std::unique_ptr<Hier>> adj;   // A^T hierarchies (built on demand)
    Csr top;                                  // whole canonical operator (per-segment batched handles)
    std::unique_ptr<Batch> batch;             // batched solve operators (built on first solve)
    double setup_seconds = 0.0;
    double adjoint_setup_seconds = 0.0;
    double resetup_seconds = 0.0;
    // numeric re-setup: input entry k -> canonical entry (or -1 for an
    // explicit zero removed at setup); empty when nothing was removed
    int64_t nnz_in = 0;
    DBuf<int32_t> canon_pos;
    std::vector<int64_t> seg_nnz;             // canonical row pointer at each segment start
};

namespace airg {
thread_local std::string g_last_error;

airg_status to_status(int st) { return static_cast<airg_status>(st); }

template <class F>
airg_status guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return AIRG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return to_status(e.status);
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

void check_opts(const airg_opts &o) {
    AIRG_REQUIRE(o.struct_size == (int32_t)sizeof(airg_opts), ST_INVALID_ARG, "opts.struct_size mismatch");
    AIRG_REQUIRE(o.poly_order >= 0 && o.poly_order + 2 <= kMaxPolyCols, ST_INVALID_ARG, "poly_order out of range");
    AIRG_REQUIRE(o.coarse_poly_order >= 0 && o.coarse_poly_order + 2 <= kMaxPolyCols, ST_INVALID_ARG,
                 "coarse_poly_order out of range");
    AIRG_REQUIRE(o.poly_sparsity_order >= 1 && o.poly_sparsity_order <= 3, ST_INVALID_ARG,
                 "poly_sparsity_order must be 1, 2 or 3");
    AIRG_REQUIRE(o.coarse_matrix_free == 0 || o.coarse_matrix_free == 1, ST_INVALID_ARG,
                 "coarse_matrix_free must be 0 or 1");
    AIRG_REQUIRE(o.time_phases == 0 || o.time_phases == 1, ST_INVALID_ARG, "time_phases must be 0 or 1");
    AIRG_REQUIRE(o.down_smooths == 0, ST_INVALID_ARG, "only up F-point smoothing is implemented");
    AIRG_REQUIRE(o.up_smooths >= 0 && o.coarse_iters >= 1, ST_INVALID_ARG, "bad smoothing counts");
    AIRG_REQUIRE(o.precond_precision == 32 || o.precond_precision == 64, ST_INVALID_ARG,
                 "precond_precision must be 32 or 64");
    AIRG_REQUIRE(o.outer == AIRG_OUTER_RICHARDSON || o.outer == AIRG_OUTER_FGMRES, ST_INVALID_ARG, "bad outer");
    AIRG_REQUIRE(o.strong_threshold >= 0.0 && std::isfinite(o.strong_threshold), ST_INVALID_ARG,
                 "bad strong_threshold");
    AIRG_REQUIRE(o.drop_R >= 0.0 && o.drop_A >= 0.0, ST_INVALID_ARG, "bad drop tolerance");
    AIRG_REQUIRE(o.pmisr_max_rounds >= 0, ST_INVALID_ARG, "bad pmisr_max_rounds");
}

// Rows [lo, hi) whose columns must stay inside [lo, hi); copied with columns
// shifted by -lo.
__global__ void k_seg_check(int32_t lo, int32_t hi, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            int32_t *__restrict__ bad) {
    int32_t i = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hi) return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] < lo || ci[k] >= hi) atomicOr(bad, 1);
}
__global__ void k_seg_rp(int32_t lo, int32_t hi, const int32_t *__restrict__ rp, int32_t *__restrict__ orp) {
    int32_t i = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (i > hi) return;
    orp[i - lo] = rp[i] - rp[lo];
}
__global__ void k_seg_ci(int64_t cnt, int32_t lo, const int32_t *__restrict__ ci, int32_t *__restrict__ oci) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cnt) oci[k] = ci[k] - lo;
}

Csr slice_segment(const Csr &A, int32_t lo, int32_t hi, hipStream_t s) {
    DBuf<int32_t> bad(1, s);
    fill_zero(bad.p, 4, s);
    int32_t m = hi - lo;
    k_seg_check<<<grid_for(m, 256), 256, 0, s>>>(lo, hi, A.rp.p, A.ci.p, bad.p);
    AIRG_LAUNCH_CHECK();
    AIRG_REQUIRE(d2h_one(bad.p, s) == 0, ST_BAD_CSR, "an entry couples two segments");
    int32_t b0 = d2h_one(A.rp.p + lo, s), b1 = d2h_one(A.rp.p + hi, s);
    Csr S;
    S.alloc(m, m, (int64_t)b1 - b0, s);
    k_seg_rp<<<grid_for((int64_t)m + 1, 256), 256, 0, s>>>(lo, hi, A.rp.p, S.rp.p);
    AIRG_LAUNCH_CHECK();
    if (S.nnz > 0) {
        k_seg_ci<<<grid_for(S.nnz, 256), 256, 0, s>>>(S.nnz, lo, A.ci.p + b0, S.ci.p);
        AIRG_LAUNCH_CHECK();
        d2d(S.v.p, A.v.p + b0, (size_t)S.nnz, s);
    }
    return S;
}

__global__ void k_strided(const double *__restrict__ src, int64_t ss, double *__restrict__ dst, int64_t ds,
                          int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i * ds] = src[i * ss];
}
void strided_copy(const double *src, int64_t ss, double *dst, int64_t ds, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_strided<<<grid_for(n, 256), 256, 0, s>>>(src, ss, dst, ds, n);
    AIRG_LAUNCH_CHECK();
}

// ------------------------------------------------------ numeric re-setup --
enum : uint32_t { RS_NONFINITE = 1, RS_ZERO_DIAG = 2, RS_OFF_PATTERN = 4 };

__global__ void k_keep_flags(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ v, int32_t *__restrict__ keep) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) keep[k] = ci[k] == i || v[k] != 0.0;
}
__global__ void k_keep_pos(int64_t nnz, const int32_t *__restrict__ keep, int32_t *__restrict__ pos) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz && !keep[k]) pos[k] = -1;
}
__global__ void k_resetup_gather(int64_t nnz, const int32_t *__restrict__ pos, const double *__restrict__ vin,
                                 double *__restrict__ vout, uint32_t *__restrict__ flags) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    int32_t p = pos[k];
    if (p >= 0) vout[p] = vin[k];
    else if (vin[k] != 0.0) atomicOr(flags, RS_OFF_PATTERN);
}
__global__ void k_resetup_check(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const double *__restrict__ v, uint32_t *__restrict__ flags) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t f = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (!isfinite(v[k])) f |= RS_NONFINITE;
        if (ci[k] == i && v[k] == 0.0) f |= RS_ZERO_DIAG;
    }
    if (f) atomicOr(flags, f);
}

// canonical_pos[k] for every input entry when setup removed explicit zeros
void record_canonical_map(airg_handle *h, int32_t n, int64_t nnz_in, const int32_t *rp, const int32_t *ci,
                          const double *v, int64_t nnz_canon, hipStream_t s) {
    h->nnz_in = nnz_in;
    if (nnz_canon == nnz_in) return;
    DBuf<int32_t> keep((size_t)nnz_in, s);
    h->canon_pos.alloc((size_t)nnz_in + 1, s);
    k_keep_flags<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, v, keep.p);
    AIRG_LAUNCH_CHECK();
    exclusive_scan(keep.p, h->canon_pos.p, nnz_in, s, false);
    k_keep_pos<<<grid_for(nnz_in, 256), 256, 0, s>>>(nnz_in, keep.p, h->canon_pos.p);
    AIRG_LAUNCH_CHECK();
}

void build_adjoint(airg_handle *h, hipStream_t s) {
    if (!h->adj.empty()) return;
    auto t0 = std::chrono::steady_clock::now();
    for (size_t p = 0; p + 1 < h->seg.size(); ++p) {
        Csr T;
        if (h->segh) {
            Csr S = slice_segment(h->segh->lv[0]->A, (int32_t)h->seg[p], (int32_t)h->seg[p + 1], s);
            T = transpose(view(S), s);
        } else {
            T = transpose(view(h->fwd[p]->L(0).A), s);
        }
        h->adj.push_back(build_hierarchy(std::move(T), h->opt, h->seeds[p], s));
    }
    AIRG_HIP(hipStreamSynchronize(s));
    h->adjoint_setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void run_solve(airg_handle *h, std::vector<std::unique_ptr<Hier>> &hs, int32_t nrhs, const double *b, double *x,
               double rtol, int32_t max_it, hipStream_t s, airg_solve_info *info) {
    AIRG_REQUIRE(nrhs >= 1, ST_INVALID_ARG, "nrhs must be >= 1");
    AIRG_REQUIRE(b && x, ST_INVALID_ARG, "null vector");
    AIRG_REQUIRE(rtol > 0.0 && max_it >= 0, ST_INVALID_ARG, "bad rtol or max_it");
    auto t0 = std::chrono::steady_clock::now();
    int its = 0;
    bool conv = true;
    double worst = 0.0;
    for (size_t p = 0; p < hs.size(); ++p) {
        Hier &H = *hs[p];
        H.s = s;
        int64_t lo = h->seg[p], m = h->seg[p + 1] - h->seg[p];
        DBuf<double> bb((size_t)m, s), xx((size_t)m, s);
        for (int32_t c = 0; c < nrhs; ++c) {
            strided_copy(b + lo * nrhs + c, nrhs, bb.p, 1, m, s);
            SolveResult r = H.opt.outer == AIRG_OUTER_FGMRES ? solve_fgmres(H, bb.p, xx.p, rtol, max_it)
                                                             : solve_richardson(H, bb.p, xx.p, rtol, max_it);
            strided_copy(xx.p, 1, x + lo * nrhs + c, nrhs, m, s);
            its = std::max(its, r.iterations);
            conv = conv && r.converged;
            worst = std::max(worst, r.rel_residual);
        }
    }
    AIRG_HIP(hipStreamSynchronize(s));
    if (info) {
        info->iterations = its;
        info->converged = conv;
        info->rel_residual = worst;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!conv) throw Error(ST_NOT_CONVERGED, "not converged within max_it");
}

bool batched_form(const airg_handle *h) {
    return h->segh || (h->fwd.size() > 1 && h->opt.outer == AIRG_OUTER_FGMRES && h->opt.precond_precision == 32);
}

// The batched solve operators for nrhs right-hand sides (built on first use).
void ensure_batch(airg_handle *h, int32_t nrhs, hipStream_t s) {
    AIRG_REQUIRE(nrhs == 1 || nrhs == 2 || nrhs == 4 || nrhs == 8, ST_INVALID_ARG,
                 "batched solve needs 1, 2, 4 or 8 right-hand sides");
    if (!h->batch || h->batch->k != nrhs) {
        h->batch.reset();
        h->batch = h->segh ? batch_from_segmented(*h->segh, nrhs, h->opt.autotune != 0, s)
                           : build_batch(h->fwd, nrhs, h->opt.autotune != 0, s);
    }
}

Hier *pick(const airg_handle *h, int32_t segment) {
    if (segment >= 0) {
        AIRG_REQUIRE((size_t)segment < h->fwd.size(), ST_INVALID_ARG, "segment out of range");
        return h->fwd[segment].get();
    }
    size_t p = (size_t)(-1 - segment);
    AIRG_REQUIRE(p < h->adj.size(), ST_INVALID_ARG, "adjoint hierarchy not built for this segment");
    return h->adj[p].get();
}

}  // namespace airg

extern "C" {

airg_status airg_default_opts(airg_opts *o) {
    if (!o) return AIRG_ERR_INVALID_ARG;
    std::memset(o, 0, sizeof *o);
    o->struct_size = (int32_t)sizeof(airg_opts);
    o->strong_threshold = 0.5;
    o->ddc_threshold = 0.9;
    o->ddc_fraction = 0.1;
    o->pmisr_max_rounds = 3;
    o->poly_order = 6;
    o->poly_sparsity_order = 1;
    o->drop_R = 0.01;
    o->drop_A = 0.001;
    o->coarse_poly_order = 12;
    o->coarse_iters = 3;
    o->truncate_n = 0;
    o->max_levels = 64;
    o->up_smooths = 2;
    o->down_smooths = 0;
    o->precond_precision = 64;
    o->outer = AIRG_OUTER_RICHARDSON;
    o->fgmres_restart = 30;
    o->seed = 0;
    o->build_adjoint = 0;
    o->onepoint_weight = 0;
    o->use_graph = 0;
    o->autotune = 0;
    o->device_bytes_cap = 0;
    o->coarse_matrix_free = 0;
    o->time_phases = 0;
    return AIRG_OK;
}

airg_status airg_setup(const airg_opts *opts, int64_t n, int64_t nnz, const int32_t *d_rowptr,
                       const int32_t *d_col, const double *d_val, int32_t nseg, const int64_t *h_seg_row_offsets,
                       const uint64_t *h_seg_seeds, void *hip_stream, airg_handle **out) {
    if (out) *out = nullptr;
    airg_handle *made = nullptr;
    airg_status st = guarded([&] {
        AIRG_REQUIRE(opts && out && d_rowptr && d_col && d_val, ST_INVALID_ARG, "null argument");
        check_opts(*opts);
        AIRG_REQUIRE(n > 0 && n < ((int64_t)1 << 31), ST_INVALID_ARG, "n out of range");
        hipStream_t s = (hipStream_t)hip_stream;
        auto t0 = std::chrono::steady_clock::now();
        struct CapScope {
            explicit CapScope(int64_t c) { set_device_cap(c); }
            ~CapScope() { set_device_cap(0); }
        } cap_scope(opts->device_bytes_cap);
        auto h = std::make_unique<airg_handle>();
        h->opt = *opts;
        h->n = n;
        int32_t ns = nseg > 1 ? nseg : 1;
        h->seg.assign(ns + 1, 0);
        if (ns > 1) {
            AIRG_REQUIRE(h_seg_row_offsets != nullptr, ST_INVALID_ARG, "segment offsets required for nseg > 1");
            for (int p = 0; p <= ns; ++p) h->seg[p] = h_seg_row_offsets[p];
            AIRG_REQUIRE(h->seg[0] == 0 && h->seg[ns] == n, ST_INVALID_ARG, "segment offsets must span 0..n");
            for (int p = 0; p < ns; ++p)
                AIRG_REQUIRE(h->seg[p + 1] > h->seg[p], ST_INVALID_ARG, "segments must be non-empty and ascending");
        } else {
            h->seg[1] = n;
        }
        h->seeds.resize(ns);
        for (int p = 0; p < ns; ++p) h->seeds[p] = h_seg_seeds ? h_seg_seeds[p] : opts->seed + (uint64_t)p;
        Csr A = canonical_copy((int32_t)n, nnz, d_rowptr, d_col, d_val, s);
        record_canonical_map(h.get(), (int32_t)n, nnz, d_rowptr, d_col, d_val, A.nnz, s);
        if (ns == 1) {
            h->seg_nnz = {0, A.nnz};
        } else {
            // the entry offsets at the segment boundaries only
            std::vector<const int32_t *> src((size_t)ns + 1);
            for (int p = 0; p <= ns; ++p) src[(size_t)p] = A.rp.p + h->seg[p];
            std::vector<int32_t> cnt((size_t)ns + 1, 1), at((size_t)ns + 1);
            read_ints(src, cnt, at.data(), s);
            for (int p = 0; p <= ns; ++p) h->seg_nnz.push_back(at[(size_t)p]);
        }
        const bool batch_solve = ns > 1 && opts->outer == AIRG_OUTER_FGMRES && opts->precond_precision == 32;
        AIRG_REQUIRE(!(batch_solve && opts->coarse_matrix_free), ST_INVALID_ARG,
                     "the batched form applies assembled coarse polynomials only");
        bool batched = batch_solve && segmented_supported(*opts);
        if (ns == 1) {
            h->fwd.push_back(build_hierarchy(std::move(A), *opts, h->seeds[0], s));
        } else if (batched) {
            check_segments(A, h->seg, s);
            h->segh = build_segmented(std::move(A), h->seg, h->seeds, *opts, s);
        } else {
            for (int p = 0; p < ns; ++p) {
                Csr S = slice_segment(A, (int32_t)h->seg[p], (int32_t)h->seg[p + 1], s);
                h->fwd.push_back(build_hierarchy(std::move(S), *opts, h->seeds[p], s));
            }
            h->top = std::move(A);
        }
        AIRG_HIP(hipStreamSynchronize(s));
        h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (opts->build_adjoint) build_adjoint(h.get(), s);
        made = h.release();
    });
    if (st == AIRG_OK) *out = made;
    return st;
}

airg_status airg_solve(airg_handle *h, int32_t nrhs, const double *d_b, double *d_x, double rtol, int32_t max_it,
                       void *hip_stream, airg_solve_info *info) {
    return guarded([&] {
        AIRG_REQUIRE(h, ST_INVALID_ARG, "null handle");
        hipStream_t s = (hipStream_t)hip_stream;
        if (!batched_form(h)) {
            run_solve(h, h->fwd, nrhs, d_b, d_x, rtol, max_it, s, info);
            return;
        }
        AIRG_REQUIRE(d_b && d_x && rtol > 0.0 && max_it >= 0, ST_INVALID_ARG, "bad argument");
        auto t0 = std::chrono::steady_clock::now();
        ensure_batch(h, nrhs, s);
        const Csr &top = h->segh ? h->segh->lv[0]->A : h->top;
        BatchResult r = solve_batch(*h->batch, top, h->seg, d_b, d_x, rtol, max_it, h->opt.fgmres_restart,
                                    h->opt.use_graph != 0, s);
        AIRG_HIP(hipStreamSynchronize(s));
        if (info) {
            info->iterations = r.iterations;
            info->converged = r.converged;
            info->rel_residual = r.worst;
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (!r.converged) throw Error(ST_NOT_CONVERGED, "not converged within max_it");
    });
}

airg_status airg_adjoint_solve(airg_handle *h, int32_t nrhs, const double *d_g, double *d_lambda, double rtol,
                               int32_t max_it, void *hip_stream, airg_solve_info *info) {
    return guarded([&] {
        AIRG_REQUIRE(h, ST_INVALID_ARG, "null handle");
        build_adjoint(h, (hipStream_t)hip_stream);
        run_solve(h, h->adj, nrhs, d_g, d_lambda, rtol, max_it, (hipStream_t)hip_stream, info);
    });
}

airg_status airg_get_stats(const airg_handle *h, airg_stats *st) {
    return guarded([&] {
        AIRG_REQUIRE(h && st, ST_INVALID_ARG, "null argument");
        std::memset(st, 0, sizeof *st);
        if (h->segh) {
            segmented_stats(*h->segh, st);
            st->setup_seconds = h->setup_seconds;
            st->device_bytes = (int64_t)dev_bytes_in_use();
            if (h->batch) {
                st->cycles_eager = h->batch->cycles_eager;
                st->cycles_graph = h->batch->cycles_graph;
            }
            return;
        }
        double n0 = 0, z0 = 0, gsum = 0, osum = 0, ssum = 0;
        for (auto &hp : h->fwd) {
            const Hier &H = *hp;
            double g, o, sc;
            complexities(H, &g, &o, &sc);
            double nn = H.lv[0]->n, zz = (double)H.lv[0]->A.nnz;
            n0 += nn;
            z0 += zz;
            gsum += g * nn;
            osum += o * zz;
            ssum += sc * zz;
            st->levels = std::max(st->levels, (int32_t)H.lv.size());
            for (int k = 0; k < AIRG_PHASE_COUNT; ++k) st->phase_seconds[k] += H.phase[k];
            st->vcycle_bytes_fp64 += vcycle_bytes(H, 8);
            st->vcycle_bytes_fp32 += vcycle_bytes(H, 4);
            const Level &T = *H.lv[0];
            st->top_spmv_bytes_fp64 += spmv_bytes(T.n, T.n, T.A.nnz, 8, false);
            const CycleCost cc = vcycle_cost(H);
            st->vcycle_nnz += cc.nnz;
            st->vcycle_index_bytes += cc.index_bytes;
            st->vcycle_vec_entries += cc.vec_entries;
            st->top_nnz += T.A.nnz;
            st->cycles_eager += H.cycles_eager;
            st->cycles_graph += H.cycles_graph;
            for (auto &lp : H.lv) st->setup_bytes += lp->setup_bytes;
        }
        st->grid_complexity = gsum / n0;
        st->operator_complexity = osum / z0;
        st->storage_complexity = ssum / z0;
        st->setup_seconds = h->setup_seconds;
        st->device_bytes = (int64_t)dev_bytes_in_use();
        st->resetup_seconds = h->resetup_seconds;
    });
}

airg_status airg_resetup(airg_handle *h, const double *d_val, void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(h && d_val, ST_INVALID_ARG, "null argument");
        AIRG_REQUIRE(!h->segh, ST_INVALID_ARG, "numeric re-setup is not available for the batched form");
        hipStream_t s = (hipStream_t)hip_stream;
        auto t0 = std::chrono::steady_clock::now();
        const int ns = (int)h->seg.size() - 1;
        const Csr &Acanon = ns == 1 ? h->fwd[0]->L(0).A : h->top;
        DBuf<double> vals((size_t)Acanon.nnz, s);
        DBuf<uint32_t> flags(1, s);
        fill_zero(flags.p, 4, s);
        if (h->canon_pos.p) {
            k_resetup_gather<<<grid_for(h->nnz_in, 256), 256, 0, s>>>(h->nnz_in, h->canon_pos.p, d_val, vals.p,
                                                                     flags.p);
            AIRG_LAUNCH_CHECK();
        } else {
            d2d(vals.p, d_val, (size_t)Acanon.nnz, s);
        }
        k_resetup_check<<<grid_for(Acanon.nr, 256), 256, 0, s>>>(Acanon.nr, Acanon.rp.p, Acanon.ci.p, vals.p,
                                                                 flags.p);
        AIRG_LAUNCH_CHECK();
        uint32_t f = d2h_one(flags.p, s);
        AIRG_REQUIRE(!(f & RS_NONFINITE), ST_NONFINITE, "new values include a non-finite value");
        AIRG_REQUIRE(!(f & RS_ZERO_DIAG), ST_ZERO_DIAG, "new values have a zero diagonal entry");
        AIRG_REQUIRE(!(f & RS_OFF_PATTERN), ST_INVALID_ARG,
                     "a new value is nonzero where setup found an explicit zero (outside the kept pattern)");
        if (ns > 1) d2d(h->top.v.p, vals.p, (size_t)h->top.nnz, s);
        for (int p = 0; p < ns; ++p) resetup_hierarchy(*h->fwd[p], vals.p + h->seg_nnz[p], s);
        for (size_t p = 0; p < h->adj.size(); ++p) {
            Csr T = transpose(view(h->fwd[p]->L(0).A), s);
            resetup_hierarchy(*h->adj[p], T.v.p, s);
        }
        h->batch.reset();
        AIRG_HIP(hipStreamSynchronize(s));
        h->resetup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    });
}

airg_status airg_vcycle(const airg_handle *h, int32_t segment, const double *d_g, double *d_e, int32_t precision,
                        void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(h && d_g && d_e, ST_INVALID_ARG, "null argument");
        AIRG_REQUIRE(!h->segh, ST_INVALID_ARG, "the batched form has no per-segment V-cycle");
        AIRG_REQUIRE(precision == 32 || precision == 64, ST_INVALID_ARG, "precision must be 32 or 64");
        Hier *H = pick(h, segment);
        H->s = (hipStream_t)hip_stream;
        apply_vcycle(*H, d_g, d_e, precision);
        AIRG_HIP(hipStreamSynchronize(H->s));
    });
}

airg_status airg_vcycle_profile(const airg_handle *h, int32_t segment, int32_t precision, int32_t reps,
                                double *h_level_seconds, int32_t max_levels, void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(h && h_level_seconds && reps > 0 && max_levels > 0, ST_INVALID_ARG, "bad argument");
        AIRG_REQUIRE(!h->segh, ST_INVALID_ARG, "the batched form has no per-segment V-cycle");
        AIRG_REQUIRE(precision == 32 || precision == 64, ST_INVALID_ARG, "precision must be 32 or 64");
        Hier *H = pick(h, segment);
        H->s = (hipStream_t)hip_stream;
        std::vector<double> t((size_t)H->nlev());
        profile_vcycle(*H, precision, reps, t.data());
        for (int l = 0; l < H->nlev() && l < max_levels; ++l) h_level_seconds[l] = t[l];
    });
}

airg_status airg_batch_vcycle_profile(airg_handle *h, int32_t nrhs, int32_t reps, double *h_level_seconds,
                                      int32_t max_levels, void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(h && h_level_seconds && reps > 0 && max_levels > 0, ST_INVALID_ARG, "bad argument");
        AIRG_REQUIRE(batched_form(h), ST_INVALID_ARG, "the handle is not in the batched form");
        hipStream_t s = (hipStream_t)hip_stream;
        ensure_batch(h, nrhs, s);
        Batch &B = *h->batch;
        std::vector<double> t(B.lv.size());
        batch_profile(B, reps, t.data(), s);
        for (size_t l = 0; l < t.size() && (int)l < max_levels; ++l) h_level_seconds[l] = t[l];
    });
}

airg_status airg_batch_vcycle(airg_handle *h, int32_t nrhs, const double *d_g, double *d_e, void *hip_stream) {
    return guarded([&] {
        AIRG_REQUIRE(h && d_g && d_e, ST_INVALID_ARG, "null argument");
        AIRG_REQUIRE(batched_form(h), ST_INVALID_ARG, "the handle is not in the batched form");
        hipStream_t s = (hipStream_t)hip_stream;
        ensure_batch(h, nrhs, s);
        batch_apply(*h->batch, d_g, d_e, h->opt.use_graph != 0, s);
        AIRG_HIP(hipStreamSynchronize(s));
    });
}

airg_status airg_get_level(const airg_handle *h, int32_t segment, int32_t level, airg_level_info *info,
                           int8_t *h_cf) {
    return guarded([&] {
        AIRG_REQUIRE(h && info, ST_INVALID_ARG, "null argument");
        if (h->segh && segment >= 0) {
            segmented_level_info(*h->segh, segment, level, info, h_cf, h->segh->s);
            return;
        }
        Hier *H = pick(h, segment);
        AIRG_REQUIRE(level >= 0 && level < H->nlev(), ST_INVALID_ARG, "level out of range");
        const Level &L = H->L(level);
        std::memset(info, 0, sizeof *info);
        info->level = level;
        info->coarsest = L.coarsest;
        info->n = L.n;
        info->n_f = L.nF;
        info->n_c = L.nC;
        info->nnz_a = L.A.nnz;
        info->nnz_aff = L.Aff.nnz;
        info->nnz_afc = L.Afc.nnz;
        info->nnz_ainv = L.Ainv.nnz;
        info->nnz_z = L.Z.nnz;
        info->nnz_w = L.W.nnz;
        info->poly_terms = L.poly.used;
        info->poly_requested = L.poly.m;
        for (int k = 0; k < L.poly.m && k < 16; ++k) info->alpha[k] = L.poly.alpha[k];
        for (int k = 0; k < AIRG_PHASE_COUNT; ++k) info->setup_seconds[k] = L.phase[k];
        info->setup_bytes = L.setup_bytes;
        if (h_cf) {
            if (L.coarsest) std::memset(h_cf, CF_F, (size_t)L.n);
            else d2h(h_cf, L.cf.p, (size_t)L.n, H->s);
        }
    });
}

airg_status airg_get_level_matrix(const airg_handle *h, int32_t segment, int32_t level, int32_t which,
                                  int32_t *h_rowptr, int32_t *h_col, double *h_val) {
    return guarded([&] {
        AIRG_REQUIRE(h, ST_INVALID_ARG, "null handle");
        if (h->segh && segment >= 0) {
            segmented_level_matrix(*h->segh, segment, level, which, h_rowptr, h_col, h_val, h->segh->s);
            return;
        }
        Hier *H = pick(h, segment);
        AIRG_REQUIRE(level >= 0 && level < H->nlev(), ST_INVALID_ARG, "level out of range");
        const Level &L = H->L(level);
        const Csr *M[6] = {&L.A, &L.Ainv, &L.Z, &L.W, &L.Aff, &L.Afc};
        AIRG_REQUIRE(which >= 0 && which < 6, ST_INVALID_ARG, "which out of range");
        const Csr &X = *M[which];
        AIRG_REQUIRE(X.rp.p != nullptr, ST_INVALID_ARG, "matrix not present on this level");
        if (h_rowptr) d2h(h_rowptr, X.rp.p, (size_t)X.nr + 1, H->s);
        if (h_col) d2h(h_col, X.ci.p, (size_t)X.nnz, H->s);
        if (h_val) d2h(h_val, X.v.p, (size_t)X.nnz, H->s);
    });
}

airg_status airg_kernel_timing(int32_t enable) {
    return guarded([&] { top_timing(enable != 0); });
}

airg_status airg_kernel_timing_read(int64_t *launches, double *bytes, double *seconds) {
    return guarded([&] {
        AIRG_REQUIRE(launches && bytes && seconds, ST_INVALID_ARG, "null argument");
        top_timing_read(launches, bytes, seconds);
    });
}

void airg_destroy(airg_handle *h) {
    if (!h) return;
    try {
        for (auto &H : h->fwd)
            if (H) (void)hipStreamSynchronize(H->s);
        if (h->segh) (void)hipStreamSynchronize(h->segh->s);
        delete h;
    } catch (...) {
    }
}

const char *airg_status_string(airg_status st) {
    switch (st) {
    case AIRG_OK: return "ok";
    case AIRG_NOT_CONVERGED: return "not converged";
    case AIRG_ERR_INVALID_ARG: return "invalid argument";
    case AIRG_ERR_BAD_CSR: return "malformed CSR matrix";
    case AIRG_ERR_ZERO_DIAG: return "zero diagonal entry";
    case AIRG_ERR_NONFINITE: return "non-finite value";
    case AIRG_ERR_OOM: return "out of device memory";
    case AIRG_ERR_HIP: return "HIP runtime error";
    case AIRG_ERR_STALL: return "iteration stalled (non-finite residual)";
    case AIRG_ERR_LIMIT: return "size exceeds a kernel limit";
    }
    return "unknown status";
}

const char *airg_last_error(void) { return airg::g_last_error.c_str(); }

}  // extern "C"
