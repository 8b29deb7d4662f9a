// Batch setup over the block-diagonal concatenation of many problems: one
// pass of the level recipe per level for all segments at once (see
// segmented.hpp), then the batch V-cycle operators, totals and per-segment
// inspection.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "cfsplit.hpp"
#include "csr.hpp"
#include "segmented.hpp"
#include "spgemm.hpp"
#include "transfer.hpp"

namespace airg {

namespace {

__global__ void k_seg_couple(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const int32_t *__restrict__ off, int nseg, int32_t *__restrict__ bad) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = seg_of(off, nseg, i);
    int32_t lo = off[p], hi = off[p + 1];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] < lo || ci[k] >= hi) {
            atomicOr(bad, 1);
            break;
        }
}

// Rows of terminal segments take the CF_T marker.
__global__ void k_mark_terminal(int32_t n, const int32_t *__restrict__ off, int nseg, const int8_t *__restrict__ term,
                                int8_t *__restrict__ cf) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (term[seg_of(off, nseg, i)]) cf[i] = CF_T;
}

template <class T>
DBuf<T> to_dev(const std::vector<T> &h, hipStream_t s) {
    DBuf<T> d(std::max<size_t>(h.size(), 1), s);
    h2d(d.p, h.data(), h.size(), s);
    return d;
}

// Row-pointer, column and FP32 value copy (the batch V-cycle reads vf only).
Csr clone_f32(const Csr &A, hipStream_t s) {
    Csr C;
    C.nr = A.nr;
    C.nc = A.nc;
    C.nnz = A.nnz;
    C.rp.alloc((size_t)A.nr + 1, s);
    C.ci.alloc((size_t)A.nnz, s);
    C.vf.alloc((size_t)A.nnz, s);
    const CopyReq req[3] = {{C.rp.p, A.rp.p, ((size_t)A.nr + 1) * sizeof(int32_t)},
                            {C.ci.p, A.ci.p, (size_t)A.nnz * sizeof(int32_t)},
                            {C.vf.p, A.vf.p, (size_t)A.nnz * sizeof(float)}};
    copy_many(req, 3, s);
    return C;
}

void finalize_seg(SegHier &H, hipStream_t s) {
    const int nl = (int)H.lv.size();
    for (auto &lp : H.lv) {
        SegLevel &L = *lp;
        L.perm.alloc((size_t)L.n, s);
        L.iperm.alloc((size_t)L.n, s);
        make_level_perm(L.n, L.nF, L.nC, L.cf.p, L.rank.p, L.perm.p, L.iperm.p, s);
    }
    std::vector<Csr *> pending;
    for (int l = 0; l < nl; ++l) {
        SegLevel &L = *H.lv[l];
        if (L.nF + L.nC == 0) continue;
        SegLevel &N = *H.lv[l + 1];
        L.AF = permute_fc_begin(view(L.A), L.fidx.p, L.nF, s);
        L.Rp = build_rp_begin(L.Z, L.nC, L.n, N.iperm.p, s);
        L.Pp = build_pp_begin(L.W, L.nF, L.nC, N.n, s);
        pending.insert(pending.end(), {&L.AF, &L.Rp, &L.Pp});
    }
    resolve_sizes(pending, s);
    for (int l = 0; l < nl; ++l) {
        SegLevel &L = *H.lv[l];
        if (L.nF + L.nC > 0) {
            SegLevel &N = *H.lv[l + 1];
            permute_fc_fill(L.AF, view(L.A), L.fidx.p, L.cf.p, L.rank.p, L.nF, s);
            build_rp_fill(L.Rp, L.Z, L.nF, N.iperm.p, s);
            build_pp_fill(L.Pp, L.W, L.nF, N.perm.p, s);
            make_f32(L.AF, s);
            make_f32(L.Rp, s);
            make_f32(L.Pp, s);
            make_f32(L.Ainv, s);
        }
        if (L.nT > 0) {
            make_f32(L.AT, s);
            make_f32(L.AinvT, s);
        }
    }
}

int64_t nnz_rows(const Csr &M, int32_t r0, int32_t nrows, hipStream_t s) {
    if (nrows <= 0 || M.rp.p == nullptr) return 0;
    int32_t a = 0, b = 0;
    d2h(&a, M.rp.p + r0, 1, s);
    d2h(&b, M.rp.p + r0 + nrows, 1, s);
    return (int64_t)b - a;
}

const SegEntry &entry(const SegHier &H, int32_t segment, int32_t level) {
    AIRG_REQUIRE(segment >= 0 && segment < H.nseg, ST_INVALID_ARG, "segment out of range");
    AIRG_REQUIRE(level >= 0 && level < (int32_t)H.lv.size(), ST_INVALID_ARG, "level out of range");
    for (const SegEntry &e : H.lv[level]->seg)
        if (e.id == segment) return e;
    throw Error(ST_INVALID_ARG, "level out of range for this segment");
}

}  // namespace

bool segmented_supported(const airg_opts &o) { return o.ddc_threshold >= 0.0; }

void check_segments(const Csr &A, const std::vector<int64_t> &seg, hipStream_t s) {
    const int nseg = (int)seg.size() - 1;
    std::vector<int32_t> off(seg.begin(), seg.end());
    DBuf<int32_t> doff = to_dev(off, s), bad(1, s);
    fill_zero(bad.p, 4, s);
    k_seg_couple<<<grid_for(A.nr, 256), 256, 0, s>>>(A.nr, A.rp.p, A.ci.p, doff.p, nseg, bad.p);
    AIRG_LAUNCH_CHECK();
    AIRG_REQUIRE(d2h_one(bad.p, s) == 0, ST_BAD_CSR, "an entry couples two segments");
}

std::unique_ptr<SegHier> build_segmented(Csr &&A0, const std::vector<int64_t> &seg,
                                         const std::vector<uint64_t> &seeds, const airg_opts &o, hipStream_t s) {
    TraceRange trace("airg batch setup");
    auto t0 = std::chrono::steady_clock::now();
    auto H = std::make_unique<SegHier>();
    H->opt = o;
    H->s = s;
    H->nseg = (int)seg.size() - 1;
    PhaseTimer tm(s, o.time_phases != 0);
    {
        auto L0 = std::make_unique<SegLevel>();
        L0->n = A0.nr;
        L0->A = std::move(A0);
        for (int p = 0; p < H->nseg; ++p) {
            SegEntry e;
            e.id = p;
            e.off = (int32_t)seg[p];
            e.n = (int32_t)(seg[p + 1] - seg[p]);
            L0->seg.push_back(e);
        }
        H->lv.push_back(std::move(L0));
    }
    const int maxl = o.max_levels > 0 ? o.max_levels : 64;
    const int m = o.poly_order + 1, mc = o.coarse_poly_order + 1;
    const int32_t min_c = std::max(o.poly_order, 1);
    Branch br(s);   // after H and tm: waits for a running job before they go
    for (int l = 0;; ++l) {
        SegLevel &L = *H->lv[l];
        const int32_t n = L.n;
        const int na = (int)L.seg.size();
        TraceRange trace_level("batch setup level %d", l);
        tm.level = l;
        std::vector<int32_t> off(na + 1);
        std::vector<uint64_t> sd(na);
        std::vector<int8_t> term(na);
        bool any_active = false;
        for (int i = 0; i < na; ++i) {
            const SegEntry &e = L.seg[i];
            off[i] = e.off;
            sd[i] = seeds[e.id];
            term[i] = (o.truncate_n > 0 && e.n <= o.truncate_n) || l == maxl - 1;
            any_active = any_active || !term[i];
        }
        off[na] = n;
        DBuf<int32_t> doff = to_dev(off, s);
        DBuf<uint64_t> dsd = to_dev(sd, s);
        L.cf.alloc((size_t)n, s);
        L.rank.alloc((size_t)n, s);
        tm.begin(AIRG_PHASE_CF);
        if (any_active) {
            StrengthGraph G = strength_graph(view(L.A), o.strong_threshold, s);
            DBuf<uint32_t> h((size_t)n, s);
            pmisr_hash_seg(n, doff.p, na, dsd.p, l, h.p, s);
            DBuf<int8_t> cf0((size_t)n, s);
            pmisr(view(L.A), G, h.p, o.pmisr_max_rounds, cf0.p, s);
            ddc(view(L.A), o.ddc_threshold, cf0.p, L.cf.p, nullptr, s);
            L.setup_bytes += split_bytes(view(L.A));
        }
        std::vector<int32_t> bnd((size_t)3 * (na + 1));
        auto mark_and_rank = [&]() {
            DBuf<int8_t> dterm = to_dev(term, s);
            k_mark_terminal<<<grid_for(n, 256), 256, 0, s>>>(n, doff.p, na, dterm.p, L.cf.p);
            AIRG_LAUNCH_CHECK();
            return cf_ranks_seg(L.cf.p, n, L.rank.p, doff.p, na, bnd.data(), s);
        };
        CfCounts c = mark_and_rank();
        if (any_active) {
            bool more = false;
            for (int i = 0; i < na; ++i) {
                if (term[i]) continue;
                int32_t nF = bnd[3 * (i + 1)] - bnd[3 * i], nC = bnd[3 * (i + 1) + 1] - bnd[3 * i + 1];
                if (nF == 0 || nC < min_c) {
                    term[i] = 1;
                    more = true;
                }
            }
            if (more) c = mark_and_rank();
        }
        tm.end();
        L.nF = c.nF;
        L.nC = c.nC;
        L.nT = c.nT;
        std::vector<int32_t> foff, toff;
        std::vector<uint64_t> fsd, tsd;
        std::vector<int> aidx, tidx;
        for (int i = 0; i < na; ++i) {
            SegEntry &e = L.seg[i];
            e.terminal = term[i] != 0;
            e.fOff = bnd[3 * i];
            e.cOff = bnd[3 * i + 1];
            e.tOff = bnd[3 * i + 2];
            if (e.terminal) {
                toff.push_back(e.tOff);
                tsd.push_back(seeds[e.id]);
                tidx.push_back(i);
            } else {
                e.nF = bnd[3 * (i + 1)] - bnd[3 * i];
                e.nC = bnd[3 * (i + 1) + 1] - bnd[3 * i + 1];
                foff.push_back(e.fOff);
                fsd.push_back(seeds[e.id]);
                aidx.push_back(i);
            }
        }
        // terminal segments: the coarse polynomial on each one's whole block
        int64_t tbytes = 0;   // their setup bytes (added once the branch has joined)
        auto terminal = [&L, &o, &toff, &tsd, &tidx, &c, mc, l](hipStream_t st, int64_t *bytes) {
            toff.push_back(c.nT);
            L.AT = extract_block(view(L.A), L.cf.p, L.rank.p, CF_T, CF_T, c.nT, c.nT, st);
            DBuf<int32_t> dtoff = to_dev(toff, st);
            DBuf<uint64_t> dtsd = to_dev(tsd, st);
            std::vector<PolyInfo> P = gmres_poly_seg(view(L.AT), toff, dtoff.p, dtsd.p, l, mc, st);
            for (size_t j = 0; j < tidx.size(); ++j) L.seg[tidx[j]].poly = P[j];
            L.AinvT = inverse_pattern(view(L.AT), o.poly_sparsity_order, st);
            poly_fixed_sparsity_seg(view(L.AT), view(L.AinvT), toff, P, L.AinvT.v.p, st);
            // extraction of the terminal block, its polynomial, the assembly
            *bytes += csr_bytes(view(L.A)) + csr_bytes(view(L.AT)) + poly_bytes(view(L.AT), mc) +
                      csr_bytes(view(L.AT)) + csr_bytes(view(L.AinvT));
        };
        if (c.nF + c.nC == 0) {   // only terminal segments are left: this thread takes them
            if (c.nT > 0) {
                tm.begin(AIRG_PHASE_POLY);
                terminal(s, &tbytes);
                tm.end();
            }
            L.setup_bytes += tbytes;
            break;
        }
        // active segments: extraction, polynomials, Z, W and the coarse operator
        auto next = std::make_unique<SegLevel>();
        // the terminal segments' polynomials, the one-point prolongator and A P
        // depend on the splitting only: the branch thread builds them on its
        // stream while this one extracts the blocks and builds the polynomials
        // and Z; the Galerkin product joins it
        Csr P, AP;
        struct Join {
            Branch *b;
            ~Join() {
                if (b) b->wait_idle();
            }
        } join{&br};
        {
            const hipStream_t bs = br.stream();
            const int32_t nF = c.nF, nC = c.nC, nT = c.nT;
            br.start([&L, &o, &tm, &P, &AP, &terminal, &tbytes, bs, nF, nC, nT, l] {
                if (nT > 0) tm.span_on(AIRG_PHASE_POLY, l, bs, [&] { terminal(bs, &tbytes); });
                tm.span_on(AIRG_PHASE_PROLONG, l, bs, [&] {
                    onepoint_prolongator(view(L.A), L.cf.p, L.rank.p, nF, nC, o.onepoint_weight, &P, &L.W, bs);
                    AP = spgemm(view(L.A), view(P), bs);
                });
            });
        }
        tm.begin(AIRG_PHASE_EXTRACT);
        L.fidx.alloc((size_t)c.nF + 1, s);
        L.cidx.alloc((size_t)c.nC + 1, s);
        cf_index_lists(L.cf.p, L.rank.p, n, L.fidx.p, L.cidx.p, s);
        Csr Acf;
        extract_fc_blocks(view(L.A), L.cf.p, L.rank.p, c.nF, c.nC, L.Aff, L.Afc, Acf, s);
        L.setup_bytes += csr_bytes(view(L.A)) + 5 * (int64_t)n + csr_bytes(view(L.Aff)) + csr_bytes(view(L.Afc)) +
                         csr_bytes(view(Acf));
        tm.begin(AIRG_PHASE_POLY);
        foff.push_back(c.nF);
        {
            DBuf<int32_t> dfoff = to_dev(foff, s);
            DBuf<uint64_t> dfsd = to_dev(fsd, s);
            std::vector<PolyInfo> P = gmres_poly_seg(view(L.Aff), foff, dfoff.p, dfsd.p, l, m, s);
            for (size_t j = 0; j < aidx.size(); ++j) L.seg[aidx[j]].poly = P[j];
            L.Ainv = inverse_pattern(view(L.Aff), o.poly_sparsity_order, s);
            poly_fixed_sparsity_seg(view(L.Aff), view(L.Ainv), foff, P, L.Ainv.v.p, s);
            L.setup_bytes += poly_bytes(view(L.Aff), m) + csr_bytes(view(L.Aff)) + csr_bytes(view(L.Ainv));
        }
        tm.begin(AIRG_PHASE_RESTRICTOR);
        {
            DropArgs dz;   // Z = -A_cf Ainv, dropped as its rows are written
            dz.tau = o.drop_R;
            dz.sign = -1.0;
            dz.keep_diag = 0;
            int64_t pz = 0;
            L.Z = spgemm_drop(view(Acf), view(L.Ainv), dz, s, &pz);
            // the product and its drop as two steps: the product written and read back whole
            L.setup_bytes += csr_bytes(view(Acf)) + csr_bytes(view(L.Ainv)) + 2 * (pz * 12 + ((int64_t)L.Z.nr + 1) * 4);
        }
        tm.end();
        join.b = nullptr;
        br.finish();
        L.setup_bytes += tbytes;
        tm.begin(AIRG_PHASE_COARSE);
        {
            Csr R = restriction_full(view(L.Z), L.fidx.p, L.cidx.p, n, s);
            DropArgs da;   // the coarse operator, dropped as its rows are written
            da.tau = o.drop_A;
            da.sign = 1.0;
            da.keep_diag = 1;
            int64_t pa = 0;
            next->A = spgemm_drop(view(R), view(AP), da, s, &pa);
            // W and P from A; A P; R from Z; R (A P); the drop of R A P
            L.setup_bytes += csr_bytes(view(L.A)) + 5 * (int64_t)n + csr_bytes(view(L.W)) + csr_bytes(view(P));
            L.setup_bytes += csr_bytes(view(L.A)) + csr_bytes(view(P)) + csr_bytes(view(AP));
            L.setup_bytes += csr_bytes(view(L.Z)) + csr_bytes(view(R));
            L.setup_bytes += csr_bytes(view(R)) + csr_bytes(view(AP)) + 3 * (pa * 12 + ((int64_t)R.nr + 1) * 4);
        }
        tm.end();
        next->n = next->A.nr;
        for (int i : aidx) {
            SegEntry e;
            e.id = L.seg[i].id;
            e.off = L.seg[i].cOff;
            e.n = L.seg[i].nC;
            next->seg.push_back(e);
        }
        H->lv.push_back(std::move(next));
    }
    tm.level = -1;
    tm.begin(AIRG_PHASE_FINALIZE);
    finalize_seg(*H, s);
    SegHier &HH = *H;
    tm.collect(H->phase, [&HH](int l, int ph, double sec) { HH.lv[l]->phase[ph] += sec; });
    H->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return H;
}

std::unique_ptr<Batch> batch_from_segmented(const SegHier &H, int k, bool tune, hipStream_t s) {
    auto B = std::make_unique<Batch>();
    B->k = k;
    B->nseg = H.nseg;
    B->coarse_iters = H.opt.coarse_iters;
    B->up_smooths = H.opt.up_smooths;
    for (auto &lp : H.lv) {
        const SegLevel &L = *lp;
        auto BL = std::make_unique<BatchLevel>();
        BL->nF = L.nF;
        BL->nC = L.nC;
        BL->nT = L.nT;
        if (L.nF + L.nC > 0) {
            BL->AF = clone_f32(L.AF, s);
            BL->Ainv = clone_f32(L.Ainv, s);
            BL->Rp = clone_f32(L.Rp, s);
            BL->Pp = clone_f32(L.Pp, s);
        }
        if (L.nT > 0) {
            BL->AT = clone_f32(L.AT, s);
            BL->AinvT = clone_f32(L.AinvT, s);
        }
        B->lv.push_back(std::move(BL));
    }
    const SegLevel &T = *H.lv[0];
    B->n = T.n;
    B->perm0.alloc((size_t)T.n, s);
    d2d(B->perm0.p, T.perm.p, (size_t)T.n, s);
    finish_batch(*B, tune, s);
    return B;
}

void segmented_stats(const SegHier &H, airg_stats *st) {
    const SegLevel &T = *H.lv[0];
    const double n0 = T.n, z0 = (double)T.A.nnz;
    double g = 0, o = 0, sc = 0;
    CycleCost c;
    const int vc = H.opt.coarse_iters;
    for (auto &lp : H.lv) {
        const SegLevel &L = *lp;
        g += L.n;
        o += (double)L.A.nnz;
        st->setup_bytes += L.setup_bytes;
        if (L.nF + L.nC > 0) {
            sc += (double)L.Ainv.nnz + (double)L.Aff.nnz + (double)L.Afc.nnz + (double)(L.Z.nnz + L.nC) +
                  (double)(L.W.nnz + L.nC);
            c.add(L.Rp.nr, L.Rp.nc, L.Rp.nnz, false, 1);
            c.add(L.Pp.nr, L.Pp.nc, L.Pp.nnz, false, 1);
            c.add(L.AF.nr, L.AF.nc, L.AF.nnz, true, H.opt.up_smooths);
            c.add(L.Ainv.nr, L.Ainv.nc, L.Ainv.nnz, true, H.opt.up_smooths);
        }
        if (L.nT > 0) {
            sc += (double)L.AinvT.nnz + (vc > 1 ? (double)L.AT.nnz : 0.0);
            c.add(L.nT, L.nT, L.AinvT.nnz, false, 1);
            c.add(L.nT, L.nT, L.AT.nnz, true, vc - 1);
            c.add(L.nT, L.nT, L.AinvT.nnz, true, vc - 1);
        }
    }
    st->levels = (int32_t)H.lv.size();
    st->grid_complexity = g / n0;
    st->operator_complexity = o / z0;
    st->storage_complexity = sc / z0;
    for (int k = 0; k < AIRG_PHASE_COUNT; ++k) st->phase_seconds[k] = H.phase[k];
    st->vcycle_bytes_fp64 = c.bytes(8, 1);
    st->vcycle_bytes_fp32 = c.bytes(4, 1);
    st->top_spmv_bytes_fp64 = spmv_bytes(T.n, T.n, T.A.nnz, 8, false);
    st->vcycle_nnz = c.nnz;
    st->vcycle_index_bytes = c.index_bytes;
    st->vcycle_vec_entries = c.vec_entries;
    st->top_nnz = T.A.nnz;
}

void segmented_level_info(const SegHier &H, int32_t segment, int32_t level, airg_level_info *info, int8_t *h_cf,
                          hipStream_t s) {
    const SegEntry &e = entry(H, segment, level);
    const SegLevel &L = *H.lv[level];
    std::memset(info, 0, sizeof *info);
    info->level = level;
    info->coarsest = e.terminal;
    info->n = e.n;
    info->n_f = e.terminal ? e.n : e.nF;
    info->n_c = e.terminal ? 0 : e.nC;
    info->nnz_a = nnz_rows(L.A, e.off, e.n, s);
    if (e.terminal) {
        info->nnz_ainv = nnz_rows(L.AinvT, e.tOff, e.n, s);
    } else {
        info->nnz_aff = nnz_rows(L.Aff, e.fOff, e.nF, s);
        info->nnz_afc = nnz_rows(L.Afc, e.fOff, e.nF, s);
        info->nnz_ainv = nnz_rows(L.Ainv, e.fOff, e.nF, s);
        info->nnz_z = nnz_rows(L.Z, e.cOff, e.nC, s);
        info->nnz_w = nnz_rows(L.W, e.fOff, e.nF, s);
    }
    info->poly_terms = e.poly.used;
    info->poly_requested = e.poly.m;
    for (int k = 0; k < e.poly.m && k < 16; ++k) info->alpha[k] = e.poly.alpha[k];
    for (int k = 0; k < AIRG_PHASE_COUNT; ++k) info->setup_seconds[k] = L.phase[k];
    info->setup_bytes = L.setup_bytes;   // the level's, over all segments
    if (h_cf) {
        if (e.terminal) std::memset(h_cf, CF_F, (size_t)e.n);
        else d2h(h_cf, L.cf.p + e.off, (size_t)e.n, s);
    }
}

void segmented_level_matrix(const SegHier &H, int32_t segment, int32_t level, int32_t which, int32_t *h_rowptr,
                            int32_t *h_col, double *h_val, hipStream_t s) {
    const SegEntry &e = entry(H, segment, level);
    const SegLevel &L = *H.lv[level];
    AIRG_REQUIRE(which >= 0 && which < 6, ST_INVALID_ARG, "which out of range");
    AIRG_REQUIRE(!e.terminal || which <= 1, ST_INVALID_ARG, "matrix not present on this level");
    const Csr *M = nullptr;
    int32_t r0 = 0, nr = 0, c0 = 0;
    switch (which) {
    case 0: M = &L.A; r0 = e.off; nr = e.n; c0 = e.off; break;
    case 1:
        if (e.terminal) {
            M = &L.AinvT; r0 = e.tOff; nr = e.n; c0 = e.tOff;
        } else {
            M = &L.Ainv; r0 = e.fOff; nr = e.nF; c0 = e.fOff;
        }
        break;
    case 2: M = &L.Z; r0 = e.cOff; nr = e.nC; c0 = e.fOff; break;
    case 3: M = &L.W; r0 = e.fOff; nr = e.nF; c0 = e.cOff; break;
    case 4: M = &L.Aff; r0 = e.fOff; nr = e.nF; c0 = e.fOff; break;
    default: M = &L.Afc; r0 = e.fOff; nr = e.nF; c0 = e.cOff; break;
    }
    std::vector<int32_t> rp((size_t)nr + 1, 0);
    if (M->rp.p) d2h(rp.data(), M->rp.p + r0, (size_t)nr + 1, s);
    const int32_t b = rp[0];
    const int64_t nz = (int64_t)rp[nr] - b;
    if (h_rowptr)
        for (int32_t i = 0; i <= nr; ++i) h_rowptr[i] = rp[i] - b;
    if (nz > 0 && h_col) {
        d2h(h_col, M->ci.p + b, (size_t)nz, s);
        for (int64_t k = 0; k < nz; ++k) h_col[k] -= c0;
    }
    if (nz > 0 && h_val) d2h(h_val, M->v.p + b, (size_t)nz, s);
}

}  // namespace airg
