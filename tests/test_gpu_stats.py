"""The solve and setup accounting of airg_get_stats / airg_get_level /
airg_vcycle_profile, through the C ABI:

* work units: the stored entries one V-cycle applies (AIRG subsection's cycle:
  [Z I] and [W; I] once, [A_ff A_fc] and Ainv once per up smooth; on the
  coarsest level Ainv once and (A, Ainv) once per further coarse iteration)
  counted independently from the oracle's replay of the same hierarchy;
* per-level setup times and setup bytes add up to the totals (single and
  batched forms); the phase times are recorded only with time_phases set;
* the cycle counters tell eager cycles from graph replays;
* the per-level V-cycle profile covers every level."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import batch as batch_problems, concat, dg_square, p0_cube

pytestmark = pytest.mark.gpu

airg = pytest.importorskip("paper_2408_08262_amd.airg")


def f_rows_nnz(A, cf):
    rp = A[0]
    lens = np.diff(np.asarray(rp, np.int64))
    return int(lens[cf == 1].sum())


@pytest.mark.parametrize("name,kw", [("dg40", {}), ("dg40_trunc", {"truncate_n": 600, "coarse_iters": 4}),
                                     ("cube12_mf", {"truncate_n": 400, "coarse_matrix_free": 1})])
def test_vcycle_work_units_match_oracle_replay(name, kw):
    P = dg_square(40) if name.startswith("dg") else p0_cube(12)
    A = airg.to_device(P.rowptr, P.col, P.val)
    h = airg.airg_setup(*A, airg.default_opts(seed=P.seed, **kw))
    st = airg.airg_get_stats(h)
    nl = st["levels"]
    alphas = [airg.airg_get_level(h, l, with_cf=False)["alpha"] for l in range(nl)]
    H = O.Hierarchy((P.rowptr, P.col, P.val), O.default_params(seed=P.seed, **kw), alphas=alphas)
    assert H.nlevels == nl
    prm = O.default_params(seed=P.seed, **kw)
    ups, vc = prm.up_smooths, prm.coarse_iters
    want = 0
    for l in range(nl):
        Al = H.matrix(l, "A")
        nnz_a = int(Al[0][-1])
        if l == nl - 1:
            if kw.get("coarse_matrix_free"):
                m = len(alphas[l])
                want += vc * (m - 1) * nnz_a + (vc - 1) * nnz_a
            else:
                nnz_i = int(H.matrix(l, "Ainv")[0][-1])
                want += nnz_i + (vc - 1) * (nnz_a + nnz_i)
            continue
        cf = H.cf(l)
        nC = int((cf == 2).sum())
        want += int(H.matrix(l, "Z")[0][-1]) + nC + int(H.matrix(l, "W")[0][-1]) + nC
        want += ups * (f_rows_nnz(Al, cf) + int(H.matrix(l, "Ainv")[0][-1]))
    assert st["vcycle_nnz"] == want
    assert st["top_nnz"] == P.nnz
    # the byte count splits into index bytes, values and vector entries
    for vb, key in ((8, "vcycle_bytes_fp64"), (4, "vcycle_bytes_fp32")):
        assert st["vcycle_index_bytes"] + vb * st["vcycle_nnz"] + vb * st["vcycle_vec_entries"] == st[key]


def test_phase_times_are_recorded_only_when_asked():
    P = dg_square(64)
    A = airg.to_device(P.rowptr, P.col, P.val)
    h = airg.airg_setup(*A, airg.default_opts(seed=P.seed))          # time_phases 0: no events
    st = airg.airg_get_stats(h)
    assert st["setup_seconds"] > 0.0 and all(v == 0.0 for v in st["phase_seconds"].values())
    assert all(v == 0.0 for v in airg.airg_get_level(h, 0, with_cf=False)["setup_seconds"].values())
    h1 = airg.airg_setup(*A, airg.default_opts(seed=P.seed, time_phases=1))
    st1 = airg.airg_get_stats(h1)
    assert st1["phase_seconds"]["cf"] > 0.0 and st1["phase_seconds"]["poly"] > 0.0
    # the events change no result: the same hierarchy either way
    for l in range(st["levels"]):
        for key in ("A", "Ainv"):
            m0 = airg.airg_get_level_matrix(h, l, key)
            m1 = airg.airg_get_level_matrix(h1, l, key)
            assert all(np.array_equal(x, y) for x, y in zip(m0[:3], m1[:3])), (l, key)
    with pytest.raises(airg.AirgError):
        airg.airg_setup(*A, airg.default_opts(seed=P.seed, time_phases=2))


def test_per_level_setup_times_add_up_and_profile_covers_levels():
    P = dg_square(96)
    A = airg.to_device(P.rowptr, P.col, P.val)
    h = airg.airg_setup(*A, airg.default_opts(seed=P.seed, time_phases=1))
    st = airg.airg_get_stats(h)
    per = {k: 0.0 for k in st["phase_seconds"]}
    tot_bytes = 0
    for l in range(st["levels"]):
        lv = airg.airg_get_level(h, l, with_cf=False)
        for k, v in lv["setup_seconds"].items():
            assert v >= 0.0
            per[k] += v
        assert lv["setup_bytes"] > 0
        tot_bytes += lv["setup_bytes"]
    assert tot_bytes == st["setup_bytes"]
    for k, v in st["phase_seconds"].items():
        if k == "finalize":
            assert per[k] == 0.0      # timed after the level loop
        else:
            assert per[k] == pytest.approx(v, rel=1e-9, abs=1e-12), k
    for prec in (32, 64):
        t = airg.airg_vcycle_profile(h, precision=prec, reps=3)
        assert len(t) == st["levels"] and all(x > 0.0 for x in t)


def test_batched_setup_bytes_add_up_over_levels():
    probs = batch_problems(count=5, lo=12, hi=40, nrhs=2)
    rp, ci, val, b, offs, seeds = concat(probs)
    A = airg.to_device(rp, ci, val)
    h = airg.airg_setup(*A, airg.default_opts(outer=airg.OUTER_FGMRES, precond_precision=32),
                        seg_offsets=offs, seg_seeds=seeds)
    st = airg.airg_get_stats(h)
    nnz0 = int(rp[-1])
    tot = 0
    for l in range(st["levels"]):
        lv = None
        for p in range(len(probs)):        # any segment present on level l reports the level's total
            try:
                lv = airg.airg_get_level(h, l, segment=p, with_cf=False)
                break
            except airg.AirgError:
                continue
        assert lv is not None, l
        assert lv["setup_bytes"] > 0, l
        tot += lv["setup_bytes"]
    assert tot == st["setup_bytes"]
    assert st["setup_bytes"] > 2 * 12 * nnz0     # the splitting alone reads A_0 twice


@pytest.mark.parametrize("use_graph", [0, 1])
def test_cycle_counters_tell_eager_from_graph(use_graph):
    P = dg_square(64)
    A = airg.to_device(P.rowptr, P.col, P.val)
    opts = airg.default_opts(seed=P.seed, outer=airg.OUTER_RICHARDSON, precond_precision=64, use_graph=use_graph)
    h = airg.airg_setup(*A, opts)
    b = torch.as_tensor(P.b, device="cuda")
    _, info = airg.airg_solve(h, b, rtol=1e-10, max_it=40, allow_not_converged=True)
    st = airg.airg_get_stats(h)
    its = info["iterations"]
    if use_graph:
        eager = min(its, 16)           # a hierarchy captures its cycle after 16 eager cycles
        assert (st["cycles_eager"], st["cycles_graph"]) == (eager, its - eager)
    else:
        assert (st["cycles_eager"], st["cycles_graph"]) == (its, 0)
