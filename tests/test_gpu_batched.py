"""Batched lockstep solve (every step one launch over all subsets, finished
subsets skipped on the device, one captured HIP graph per restart cycle,
replayed with host synchronisation between replays) against the same subsets
solved one by one, and the batched solutions against the oracle's dense
residual.

The batched kernels run the per-subset arithmetic unchanged (grids only grow
to the largest subset, with per-subset guards; every reduction keeps its
order), so iteration counts must agree exactly and the solutions to rounding
of the final fp64 reconstruction (1e-10 relative)."""
import sys

import numpy as np
import pytest

from oracle import lowrank as olr
from workloads import config

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "no GPU"
    return t


@pytest.fixture(scope="module")
def L():
    from paper_2008_10275_amd import lrcheb
    return lrcheb


@pytest.fixture(scope="module")
def ctx(torch, L):
    return L.Context(0)


@pytest.fixture(scope="module")
def c3(L, ctx):
    """The uneven-subset workload at grid 65 (subset sizes 4..30, 16 subsets,
    each with its own perturbed convection coefficients)."""
    cfg = config("c3", small=True)
    f = cfg["f"]
    subs = []
    for sub in cfg["subsets"]:
        ops = L.Operators(ctx, sub["ops"].K)
        m = sub["d"].shape[1]
        p = L.Problem(ops, sub["d"], f[:, None], np.ones((m, 1)))
        p.precondition()
        subs.append(dict(ops=ops, prob=p, K=sub["ops"].K, d=sub["d"]))
    return cfg, subs


def _dense(sol):
    U, s, V = sol
    return U @ np.diag(s) @ V.T


def _kw(L, precision, recurrence="direction"):
    prec = {"fp64": L.LRC_FP64, "mixed": L.LRC_MIXED_FP32, "dir": L.LRC_MIXED_FP32_DIR}[precision]
    rec = {"direction": L.LRC_CHEB_DIRECTION, "three_term": L.LRC_CHEB_THREE_TERM}[recurrence]
    return dict(rank_cap=30, trunc_tol=1e-8, res_tol=1e-6, init=L.LRC_INIT_MEDIAN,
                precision=prec, verify_fp64=1, recurrence=rec)


@pytest.mark.parametrize("recurrence", ["direction", "three_term"])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "dir"])
def test_batched_matches_subset_solves(torch, L, ctx, c3, precision, recurrence):
    """The subsets stop at different steps of a cycle, so in the three-term
    form their iterates end in either of its two buffers."""
    cfg, subs = c3
    kw = _kw(L, precision, recurrence)
    seq = []
    for j, sb in enumerate(subs):
        say("sequential", precision, recurrence, "subset", j, "m", sb["d"].shape[1])
        code, info = sb["prob"].solve(**kw)
        assert code == 0, (j, info)
        seq.append((info, _dense(sb["prob"].solution())))
    say("batched", precision, recurrence, len(subs), "subsets")
    code, infos = L.solve_batched([sb["prob"] for sb in subs], **kw)
    assert code == 0, infos
    f = cfg["f"]
    for j, sb in enumerate(subs):
        info = infos[j]
        say("subset", j, "iters", info["iters"], seq[j][0]["iters"], "relres", info["relres"])
        assert info["status"] == 0 and info["relres"] <= 1e-6
        assert info["iters"] == seq[j][0]["iters"]
        assert info["refinements"] == seq[j][0]["refinements"]
        X = _dense(sb["prob"].solution())
        Xs = seq[j][1]
        assert np.linalg.norm(X - Xs) <= 1e-10 * np.linalg.norm(Xs)
        if j in (0, 1, 6):   # oracle dense residual on a few subsets (sizes 4, 30, 27)
            Fd = np.outer(f, np.ones(sb["d"].shape[1]))
            assert olr.relres_dense(sb["K"], sb["d"], X, Fd) <= 1.01e-6


def test_batched_mixed_structures(torch, L, ctx, c3):
    """Two subsets whose preconditioners have different supernode structures
    (leaf sizes 64 and 8) take the per-subset preconditioner launches inside
    the batch; a single-problem batch is the degenerate case."""
    cfg, subs = c3
    kw = _kw(L, "mixed")
    a, b = subs[3], subs[9]
    b["prob"].precondition(leaf_size=8)
    try:
        ref = []
        for sb in (a, b):
            code, info = sb["prob"].solve(**kw)
            assert code == 0
            ref.append((info, _dense(sb["prob"].solution())))
        say("batched, two structures")
        code, infos = L.solve_batched([a["prob"], b["prob"]], **kw)
        assert code == 0
        for (info0, X0), info, sb in zip(ref, infos, (a, b)):
            assert info["iters"] == info0["iters"]
            X = _dense(sb["prob"].solution())
            assert np.linalg.norm(X - X0) <= 1e-10 * np.linalg.norm(X0)
        say("batched, one problem")
        code, infos = L.solve_batched([a["prob"]], **kw)
        assert code == 0 and infos[0]["iters"] == ref[0][0]["iters"]
    finally:
        b["prob"].precondition()


def test_batched_rejects_unbounded_cycle(torch, L, ctx, c3):
    _, subs = c3
    with pytest.raises(L.LrcError):
        L.solve_batched([subs[0]["prob"]], **dict(_kw(L, "fp64"), restart=0))


@pytest.mark.parametrize("precision", ["fp64", "mixed", "dir"])
def test_graph_replay_matches_eager_launches(torch, L, ctx, c3, precision):
    """The captured graphs (replayed several times per solve, with host reads
    of the device flags between replays) against the same steps launched
    directly: identical iteration counts and solutions."""
    _, subs = c3
    probs = [subs[j]["prob"] for j in (1, 4, 8)]
    kw = _kw(L, precision)
    code_e, inf_e = L.solve_batched(probs, **dict(kw, eager=1))
    X_e = [_dense(p.solution()) for p in probs]
    code_g, inf_g = L.solve_batched(probs, **kw)
    X_g = [_dense(p.solution()) for p in probs]
    assert code_e == 0 and code_g == 0
    for a, b, xe, xg in zip(inf_e, inf_g, X_e, X_g):
        assert a["iters"] == b["iters"] and a["median_iters"] == b["median_iters"]
        assert np.linalg.norm(xe - xg) <= 1e-12 * np.linalg.norm(xe)


@pytest.mark.parametrize("restart", [5, 3])
@pytest.mark.parametrize("precision", ["fp64", "dir"])
def test_half_cycles_three_term_odd_restart(torch, L, ctx, c3, precision, restart):
    """A cycle runs as two captured halves, the second skipped when every
    running subset's measured rate says it stops within the first; with an
    odd cycle the three-term iterate ends a cycle in the second buffer and is
    copied back.  Graph replays against direct launches and against the
    subsets solved one by one: identical iteration counts and solutions."""
    _, subs = c3
    probs = [subs[j]["prob"] for j in (0, 2, 5, 7)]
    kw = dict(_kw(L, precision, "three_term"), restart=restart)
    say("half cycles", precision, "restart", restart)
    code_e, inf_e = L.solve_batched(probs, **dict(kw, eager=1))
    X_e = [_dense(p.solution()) for p in probs]
    code_g, inf_g = L.solve_batched(probs, **kw)
    X_g = [_dense(p.solution()) for p in probs]
    assert code_e == 0 and code_g == 0
    for j, p in enumerate(probs):
        code, info = p.solve(**kw)
        assert code == 0
        X = _dense(p.solution())
        say("subset", j, "iters", inf_g[j]["iters"], inf_e[j]["iters"], info["iters"])
        assert inf_g[j]["iters"] == inf_e[j]["iters"] == info["iters"]
        assert inf_g[j]["relres"] <= 1e-6
        assert np.linalg.norm(X_g[j] - X_e[j]) <= 1e-12 * np.linalg.norm(X_e[j])
        assert np.linalg.norm(X_g[j] - X) <= 1e-10 * np.linalg.norm(X)
