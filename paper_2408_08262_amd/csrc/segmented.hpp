// Batch setup: the AIRG level recipe run once per level over the block-
// diagonal concatenation of many independent problems (segments).  Every
// row-local step (strength, PMISR rounds, DDC, extraction, SpGEMM, drops,
// one-point prolongator) runs on the concatenated operator in one launch per
// step; the steps that depend on the problem -- PMISR keys and the random
// vector (seed and index within the segment), the GMRES polynomial (its own
// column scaling, R factor and coefficients) and termination -- are taken per
// segment, so that every segment's hierarchy is the one its own setup would
// build.  A segment whose hierarchy ends at level l has its rows marked
// terminal (CF_T) there: they take the coarse polynomial and leave the level
// recursion.  The levels come out directly in the batch V-cycle layout.
#pragma once
#include "batch.hpp"
#include "hierarchy.hpp"

namespace airg {

struct SegEntry {
    int32_t id = 0;                      // batch segment
    int32_t off = 0, n = 0;              // rows off .. off+n-1 of the level operator
    int32_t nF = 0, nC = 0;              // split counts (active segments)
    int32_t fOff = 0, cOff = 0, tOff = 0;  // first F / C / terminal rank of the segment
    bool terminal = false;
    PolyInfo poly;                       // F-block polynomial, or the coarse one when terminal
};

struct SegLevel {
    int32_t n = 0, nF = 0, nC = 0, nT = 0;
    Csr A;                               // segments present, concatenated in batch order
    DBuf<int8_t> cf;                     // CF_F, CF_C or CF_T
    DBuf<int32_t> rank, fidx, cidx;
    Csr Aff, Afc, Ainv, Z, W;            // active part
    Csr AT, AinvT;                       // terminal part (rows in terminal rank order)
    std::vector<SegEntry> seg;
    DBuf<int32_t> perm, iperm;           // natural <-> level order [F | C | T]
    Csr AF, Rp, Pp;                      // solve operators of the active part (level order)
    double phase[AIRG_PHASE_COUNT] = {};  // setup device time of the level (all segments) by phase
    int64_t setup_bytes = 0;             // algorithmic bytes of the level's setup steps (all segments)
};

struct SegHier {
    airg_opts opt{};
    hipStream_t s = nullptr;
    int nseg = 0;
    std::vector<std::unique_ptr<SegLevel>> lv;
    double phase[AIRG_PHASE_COUNT] = {};
    double setup_seconds = 0.0;
};

// Whether the batch setup covers these options (direct DDC threshold).
bool segmented_supported(const airg_opts &o);

// Checks that no entry of A couples two segments (throws ST_BAD_CSR).
void check_segments(const Csr &A, const std::vector<int64_t> &seg, hipStream_t s);

// Builds the batch hierarchy of the canonical block-diagonal A0 (takes
// ownership); seg holds nseg + 1 row offsets, seeds one seed per segment.
std::unique_ptr<SegHier> build_segmented(Csr &&A0, const std::vector<int64_t> &seg,
                                         const std::vector<uint64_t> &seeds, const airg_opts &o, hipStream_t s);

// Batch V-cycle operators for k right-hand sides (FP32 copies).
std::unique_ptr<Batch> batch_from_segmented(const SegHier &H, int k, bool tune, hipStream_t s);

// Totals over all segments.
void segmented_stats(const SegHier &H, airg_stats *st);

// One segment's view of level l (host copies); throws ST_INVALID_ARG when the
// segment's hierarchy has fewer levels.
void segmented_level_info(const SegHier &H, int32_t segment, int32_t level, airg_level_info *info, int8_t *h_cf,
                          hipStream_t s);
void segmented_level_matrix(const SegHier &H, int32_t segment, int32_t level, int32_t which, int32_t *h_rowptr,
                            int32_t *h_col, double *h_val, hipStream_t s);

}  // namespace airg
