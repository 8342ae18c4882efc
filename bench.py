#!/usr/bin/env python3
"""Time to relative residual 1e-6 of the low-rank ChebyshevT matrix-equation
solve on one MI355X (Benner, Richter, Weinhandl, arXiv 2008.10275: one Newton
step on a parameter subset, Sec. 3.4 and Algorithm 1; ChebyshevT, Sec. 4.1).

Workload (default): the 3-term stencil problem on a 513 x 513 grid
(n = 263,169), m = 1,000 random parameters, rank cap 40, truncation tolerance
1e-8, mixed precision (--precision dir: fp64 iterate, residual SpMM and
truncations, fp32 preconditioner solves) and the three-term form of the
Chebyshev recurrence (--recurrence; one truncation per update instead of the
direction form's two).  A step is one complete solve: median-parameter
initial guess, ChebyshevT, and the fp64 entry-wise residual that confirms
relres <= 1e-6.  The line also times plain fp64 in the direction form, fp64
in the timed solve's recurrence, the fp32-inner refinement form and the other
recurrence.  The preconditioner factorisation is set-up and is timed
separately.

--workload c3 times the batched form instead: 16 parameter subsets of uneven
size (20..300, 2,000 parameters in all), each with its own perturbed
convection coefficients, on a 257 x 257 grid (n = 66,049), rank cap 30; a
step is one lockstep solve of all subsets (lrc_solve_batched, mixed precision,
each restart cycle replayed from captured HIP graphs), compared with the 16
subsets solved one after another in plain FP64.

Prints one JSON line.  Per-kernel times come from HIP events recorded by the
library on the stream each kernel runs on (lrc_profile_*), the algorithmic
work per launch from the library's work models; the CPU baseline is the FP64
oracle solving the same problem on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK = {"hbm": 8000.0,                         # GB/s
        "mfma.f32": 157.3, "mfma.f64": 78.6}   # TFLOP/s (dense)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5r"],
                    help="c5r: the 3D workload at 48^3 and rank cap 40")
    ap.add_argument("--small", action="store_true", help="reduced grid (tests)")
    ap.add_argument("--precision", default="dir", choices=["mixed", "dir", "fp64", "bf16gram"],
                    help="mixed: fp32 ChebyshevT in fp64 refinement; dir: fp64 iterate and "
                         "residual with fp32 preconditioner solves and directions; bf16gram: "
                         "mixed with bf16 first-pass Gram products")
    ap.add_argument("--recurrence", default="three_term", choices=["direction", "three_term"],
                    help="form of the Chebyshev recurrence of the timed solve")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-profile", action="store_true", help="no event timing in the timed region")
    ap.add_argument("--eager", action="store_true",
                    help="timed steps launch every kernel directly (no graph replay)")
    ap.add_argument("--no-orthogonality", action="store_true",
                    help="skip the max |Q^T Q - I| report (profiled runs)")
    ap.add_argument("--no-spmm-roofline", action="store_true",
                    help="skip the SpMM-alone measurement (profiler runs of the solve)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    return ap.parse_args()


def problem_setup(L, name, small):
    from workloads import config
    cfg = config(name, small=small)
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    ctx = L.Context(0)
    ops = L.Operators(ctx, K)
    prob = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    t0 = time.perf_counter()
    prob.precondition()
    setup_s = time.perf_counter() - t0
    return cfg, ctx, ops, prob, setup_s


def batched_setup(L, small):
    from workloads import config
    cfg = config("c3", small=small)
    ctx = L.Context(0)
    f = cfg["f"]
    subs = []
    t0 = time.perf_counter()
    for sub in cfg["subsets"]:
        ops = L.Operators(ctx, sub["ops"].K)
        m = sub["d"].shape[1]
        p = L.Problem(ops, sub["d"], f[:, None], np.ones((m, 1)))
        p.precondition()
        subs.append((ops, p))
    return cfg, ctx, subs, time.perf_counter() - t0


def batched_solve(L, probs, opts, res_tol):
    code, infos = L.solve_batched(probs, opts)
    bad = [i for i in infos if i["status"] != 0 or not i["relres"] <= res_tol]
    if code != 0 or bad:
        raise RuntimeError(f"batched solve did not reach {res_tol}: status {code}, {bad[:2]}")
    return infos


def main_batched(a, L, torch):
    cfg, ctx, subs, setup_s = batched_setup(L, a.small)
    probs = [p for _, p in subs]
    res_tol = cfg["res_tol"]
    opts = solve_opts(L, cfg, a.precision, recurrence=a.recurrence)
    for _ in range(max(1, a.warmup)):
        batched_solve(L, probs, opts, res_tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        infos = batched_solve(L, probs, opts, res_tol)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / a.steps
    # the same subsets one after another, plain FP64
    seq = None
    if not a.no_fp64_compare:
        o64 = solve_opts(L, cfg, "fp64")
        for p in probs:
            one_solve(p, o64, res_tol)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        reps = max(1, min(a.steps, 3))
        for _ in range(reps):
            seq_infos = [one_solve(p, o64, res_tol) for p in probs]
        torch.cuda.synchronize()
        seq = dict(seconds=(time.perf_counter() - t1) / reps,
                   iters=[i["iters"] for i in seq_infos],
                   max_relres=max(i["relres"] for i in seq_infos))
    # kernel table of the batched solve (eager launches, HIP events)
    oe = L.default_opts(**{f: getattr(opts, f) for f, _ in opts._fields_})
    oe.eager = 1
    ktab = {} if a.no_profile else profiled(L, lambda: batched_solve(L, probs, oe, res_tol),
                                            a.steps, torch)
    roof = roofline_of(ktab, "HIP events on the library stream around every launch, in a "
                             "repeat of the batched solve with eager launches")
    cpu = None
    if not a.no_cpu:
        # the oracle on a bounded sample: two of the subsets, scaled to all 16
        # by their parameter counts
        subs_cfg = cfg["subsets"]
        pick = [0, 5]
        secs, its = 0.0, []
        for j in pick:
            t, it = cpu_oracle_solve(subs_cfg[j]["ops"].K, subs_cfg[j]["d"], cfg["f"],
                                     cfg["rank_cap"], cfg["trunc_tol"], res_tol)
            secs += t
            its.append(it)
        msample = sum(subs_cfg[j]["d"].shape[1] for j in pick)
        mall = sum(s_["d"].shape[1] for s_ in subs_cfg)
        cpu = dict(value=secs * mall / msample, unit="s", cores=int(blas_threads()),
                   kind="oracle", host=host_info(),
                   sample=(f"oracle solves of subsets {pick} ({msample} of {mall} parameters, "
                           f"{its} iterations, {secs:.2f} s), scaled to all subsets by "
                           f"parameter count; SuperLU single-threaded, BLAS on "
                           f"{blas_threads()} threads"))
    n = cfg["base_ops"].n
    sizes = cfg["sizes"]
    line = {
        "metric": "time to rel. residual 1e-6 (s), all subsets",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": (f"{len(sizes)} parameter subsets of sizes {min(sizes)}..{max(sizes)} "
                                f"({sum(sizes)} parameters), each with its own perturbed "
                                f"convection coefficients, {int(round(np.sqrt(n)))}x"
                                f"{int(round(np.sqrt(n)))} grid, n={n}, rank cap "
                                f"{cfg['rank_cap']}, relres {res_tol:g}, batched lockstep solve"),
                   "n": int(n), "subsets": len(sizes), "m_total": int(sum(sizes)),
                   "rank_cap": cfg["rank_cap"], "trunc_tol": cfg["trunc_tol"],
                   "precision": a.precision, "recurrence": a.recurrence},
        "result": {"iters": [i["iters"] for i in infos],
                   "max_relres_fp64": max(i["relres"] for i in infos),
                   "setup_s": setup_s},
        "sequential_fp64": seq,
        "speedup_vs_sequential_fp64": (seq["seconds"] / sec) if seq else None,
        "roofline": roof,
        "kernels": ktab,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main_surrogate(a, L, torch):
    """Learned initial guess (surrogate-seeded solve) against the median one on
    held-out parameters.  Untimed set-up: the training subset is solved on the
    GPU, its solution gives the POD basis U0 and coefficients (GPU
    truncation), the network is trained by the library's kernels.  Timed: for
    the held-out subset, network inference + X0 = U0 C^T + ChebyshevT to 1e-6
    (learned), against the median-parameter solve + ChebyshevT (median), both
    in the chosen precision, and the plain FP64 median form."""
    from workloads import config, mlp_init
    cfg = config("c4", small=a.small)
    K, f = cfg["ops"].K, cfg["f"]
    dtr, dte = cfg["d_train"], cfg["d_test"]
    r = cfg["basis_rank"]
    ctx = L.Context(0)
    ops = L.Operators(ctx, K)
    n = K[0].shape[0]

    def prob(d):
        p = L.Problem(ops, d, f[:, None], np.ones((d.shape[1], 1)))
        p.precondition()
        return p

    ptr, pte = prob(dtr), prob(dte)
    res_tol = cfg["res_tol"]
    base = dict(rank_cap=cfg["rank_cap"], trunc_tol=cfg["trunc_tol"], res_tol=res_tol,
                verify_fp64=1, recurrence={"direction": L.LRC_CHEB_DIRECTION,
                                           "three_term": L.LRC_CHEB_THREE_TERM}[a.recurrence])
    code, _ = ptr.solve(L.default_opts(**base, init=L.LRC_INIT_MEDIAN, precision=L.LRC_FP64))
    if code != 0:
        raise RuntimeError("training snapshots did not converge")
    U, sv, V = ptr.solution()
    k = U.shape[1]
    ld = (k + 7) // 8 * 8
    Ud = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    Ud[:, :k] = torch.from_numpy(U).cuda()
    Vd = torch.zeros((V.shape[0], ld), dtype=torch.float64, device="cuda")
    Vd[:, :k] = torch.from_numpy(V).cuda()
    Xtr = torch.from_numpy(np.ascontiguousarray(dtr[1:].T)).cuda()
    Xte = torch.from_numpy(np.ascontiguousarray(dte[1:].T)).cuda()

    def surrogate(tol):
        """POD basis of the snapshots (rank cap r, tail cut at tol) and the
        network trained on its coefficients."""
        U0 = torch.zeros((n, 32), dtype=torch.float64, device="cuda")
        V0 = torch.zeros((V.shape[0], 32), dtype=torch.float64, device="cuda")
        s0, rr = L.truncate_dev(ctx, Ud, sv, Vd, r, tol, U0, V0)
        Ctr = (V0[:, :rr] * torch.from_numpy(s0).cuda()).contiguous()
        net = L.MLP(ctx, mlp_init(11, sizes=(2, 64, 64, rr)))
        net.fit_scaling(Xtr, Ctr)
        hist = net.train(Xtr, Ctr, 2000, lr=3e-3)
        return U0[:, :rr].contiguous(), rr, net, hist

    # POD basis truncated at the solver's own tolerance (modes below it are
    # rounding noise that would only widen the residual), and the same basis
    # kept at the configured rank r (tail cut at zero)
    U0r, rr, net, hist = surrogate(cfg["trunc_tol"])
    U0w, rw, netw, histw = surrogate(0.0)
    prec = {"mixed": L.LRC_MIXED_FP32, "dir": L.LRC_MIXED_FP32_DIR, "fp64": L.LRC_FP64}[a.precision]
    o_l = L.default_opts(**base, init=L.LRC_INIT_GIVEN, precision=prec)
    o_j = L.default_opts(**base, init=L.LRC_INIT_GIVEN_JUDGED, precision=prec)
    o_m = L.default_opts(**base, init=L.LRC_INIT_MEDIAN, precision=prec)
    o_p = L.default_opts(**dict(base, recurrence=L.LRC_CHEB_DIRECTION), init=L.LRC_INIT_MEDIAN,
                         precision=L.LRC_FP64)

    def learned(o=o_l, U=U0r, nt=net):
        C = nt.predict(Xte)
        code, info = pte.solve_x0_dev(U, C, opts=o)
        return code, info

    def median(o):
        return pte.solve(o)

    def timed(fn):
        for _ in range(max(1, a.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            code, info = fn()
        torch.cuda.synchronize()
        if code != 0 or not info["relres"] <= res_tol:
            raise RuntimeError(f"solve did not reach {res_tol}: {code} {info}")
        return (time.perf_counter() - t0) / a.steps, info

    t_l, i_l = timed(learned)
    t_j, i_j = timed(lambda: learned(o_j))
    t_w, i_w = timed(lambda: learned(o_l, U0w, netw))
    t_m, i_m = timed(lambda: median(o_m))
    t_p, i_p = timed(lambda: median(o_p))
    ktab, roof, cpu = {}, None, None
    if not a.no_profile:
        ol_e = L.default_opts(**base, init=L.LRC_INIT_GIVEN, precision=prec, eager=1)
        ktab = profiled(L, lambda: learned(ol_e), a.steps, torch)
        roof = roofline_of(ktab, "HIP events on the library stream around every launch, in a "
                                 "repeat of the learned-guess solve with eager launches")
    if not a.no_cpu:
        secs, its = cpu_oracle_solve(K, dte, f, cfg["rank_cap"], cfg["trunc_tol"], res_tol)
        cpu = dict(value=secs, unit="s", cores=int(blas_threads()), kind="oracle",
                   host=host_info(),
                   sample=(f"one oracle solve of the held-out set from the median guess "
                           f"(n={n}, m={dte.shape[1]}, {its} iterations); SuperLU "
                           f"single-threaded, BLAS on {blas_threads()} threads"))
    line = {
        "metric": "time to rel. residual 1e-6 (s), learned initial guess",
        "value": t_l, "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": t_l * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"learned initial guess on {dte.shape[1]} held-out parameters, "
                                f"network 2-64-64-{rr} trained on {dtr.shape[1]} GPU solutions "
                                f"(POD rank {rr}), 3-term stencil equation on a "
                                f"{int(round(np.sqrt(n)))}x{int(round(np.sqrt(n)))} grid, n={n}"),
                   "n": int(n), "m_train": int(dtr.shape[1]), "m_test": int(dte.shape[1]),
                   "rank_cap": cfg["rank_cap"], "pod_rank": int(rr), "precision": a.precision,
                   "recurrence": a.recurrence},
        "result": {"learned": dict(seconds=t_l, iters=i_l["iters"], relres=i_l["relres"]),
                   "learned_judged": dict(seconds=t_j, iters=i_j["iters"], relres=i_j["relres"],
                                          fallback_cols=i_j["median_fallback_cols"],
                                          fallback_rate=i_j["median_fallback_cols"] /
                                          dte.shape[1]),
                   "learned_rank_r": dict(seconds=t_w, iters=i_w["iters"], relres=i_w["relres"],
                                          pod_rank=int(rw)),
                   "median": dict(seconds=t_m, iters=i_m["iters"], relres=i_m["relres"],
                                  median_iters=i_m["median_iters"]),
                   "fp64_median": dict(seconds=t_p, iters=i_p["iters"], relres=i_p["relres"]),
                   "train_loss": [float(hist[0]), float(hist[-1])]},
        "speedup_vs_median": t_m / t_l,
        "speedup_vs_fp64_median": t_p / t_l,
        "roofline": roof,
        "kernels": ktab,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def solve_opts(L, cfg, precision, eager=0, recurrence="direction"):
    return L.default_opts(rank_cap=cfg["rank_cap"], trunc_tol=cfg["trunc_tol"],
                          res_tol=cfg["res_tol"], init=L.LRC_INIT_MEDIAN, verify_fp64=1,
                          precision={"mixed": L.LRC_MIXED_FP32, "dir": L.LRC_MIXED_FP32_DIR,
                                     "fp64": L.LRC_FP64,
                                     "bf16gram": L.LRC_MIXED_BF16GRAM}[precision],
                          eager=eager,
                          recurrence={"direction": L.LRC_CHEB_DIRECTION,
                                      "three_term": L.LRC_CHEB_THREE_TERM}[recurrence])


def workload_name(cfg, n, m):
    if cfg["ops"].dim == 3:
        N = cfg["ops"].N
        return (f"3-term 3D stencil equation (7-point upwind convection-diffusion + 27-point "
                f"solid-cube Laplacian and grad-div), {N}^3 grid, n={n}, m={m} parameters, rank "
                f"cap {cfg['rank_cap']} (reduced from 102^3 and cap 60: the truncation holds "
                f"128 columns), relres {cfg['res_tol']:g}")
    N = int(round(np.sqrt(n)))
    return (f"3-term 2D stencil equation (upwind convection-diffusion + solid-box Laplacian "
            f"and grad-div), {N}x{N} grid, n={n}, m={m} parameters, rank cap "
            f"{cfg['rank_cap']}, relres {cfg['res_tol']:g}")


def one_solve(prob, opts, res_tol):
    code, info = prob.solve(opts)
    if code != 0 or not info["relres"] <= res_tol:
        raise RuntimeError(f"solve did not reach {res_tol}: status {code}, info {info}")
    return info


TRAFFIC = os.path.join(HERE, "profiles", "hbm_traffic_c2_dir.md")


def measured_traffic(kernel):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated), or None when there is none
    or the kernel's source file changed since the counters were taken."""
    import hashlib
    try:
        lines = open(TRAFFIC).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) == 6 and cells[0] == kernel and ":" in cells[5]:
            fname, digest = cells[5].split(":")
            path = os.path.join(HERE, "paper_2008_10275_amd", "csrc", fname)
            try:
                now = hashlib.sha256(open(path, "rb").read()).hexdigest()[:12]
            except OSError:
                return None
            return float(cells[4]) if now == digest else None
    return None


KTIMES = os.path.join(HERE, "profiles", "solve_dir_c2_kernels.md")


def _source_ok(cell):
    import hashlib
    if ":" not in cell:
        return False
    fname, dig = cell.split(":")
    try:
        now = hashlib.sha256(open(os.path.join(HERE, "paper_2008_10275_amd", "csrc", fname),
                                  "rb").read()).hexdigest()[:12]
    except OSError:
        return False
    return now == dig


def rocprof_avg_us(kernel):
    """Average launch duration of a kernel class in the committed rocprofv3
    kernel-trace summary, or None when there is none or the kernel's source
    changed since the trace was taken."""
    try:
        lines = open(KTIMES).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) == 6 and cells[0] == kernel and _source_ok(cells[5]):
            return float(cells[2])
    return None


def kernel_table(prof_work, prof_time, steps):
    """Per class: ms per step, launches per step, achieved rate, fraction of peak."""
    out = {}
    for name, t in prof_time.items():
        if t["count"] == 0:
            continue
        w = prof_work.get(name, {})
        row = dict(ms_per_step=t["ms"] / steps, launches_per_step=t["count"] / steps)
        if w.get("unit") and w.get("count", 0) == t["count"] / steps and t["ms"] > 0:
            avg_ms = t["ms"] / t["count"]
            work_per_launch = w["work"] / w["count"]
            if w["unit"] == "B":
                bound, unit, ach = "hbm", "GB/s", work_per_launch / (avg_ms * 1e-3) / 1e9
                peak = PEAK["hbm"]
            else:
                dt = name.split(".")[1]
                bound, unit = "mfma", "TFLOP/s"
                ach = work_per_launch / (avg_ms * 1e-3) / 1e12
                peak = PEAK["mfma." + dt]
            row.update(bound=bound, achieved=ach, peak=peak, unit=unit, frac=ach / peak,
                       work_per_launch=work_per_launch, work_unit=w["unit"],
                       avg_launch_us=avg_ms * 1e3)
        out[name] = row
    return out


def host_info():
    """Host CPU facts for the baseline: logical CPUs, the CPUs this process may
    run on, and the model name."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return dict(nproc=os.cpu_count() or 1, cpus_available=avail, cpu_model=model)


_DIRECT = {}


def _direct_column(j):
    """One parameter column solved the standard way (Sec. 5.1's reference
    method for a linear problem: factorise A_j and solve), in a worker."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle import lowrank as olr
    K, d, f = _DIRECT["K"], _DIRECT["d"], _DIRECT["f"]
    t0 = time.perf_counter()
    spla.splu(sp.csc_matrix(olr.column_operator(K, d, j))).solve(f)
    return time.perf_counter() - t0


def consecutive_direct(cfg, workers, sample):
    """The consecutive direct baseline: every column factorised and solved on
    its own (SuperLU), the m columns spread over a pool of `workers`
    processes.  Timed on `sample` columns (the pool's wall time) and scaled to
    all m columns."""
    import multiprocessing as mp
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    _DIRECT.update(K=K, d=d, f=f)
    cols = np.linspace(0, m - 1, min(sample, m)).astype(int).tolist()
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_direct_column, cols[:workers])          # warm the workers
        t0 = time.perf_counter()
        per = pool.map(_direct_column, cols)
        wall = time.perf_counter() - t0
    return dict(value=wall * m / len(cols), unit="s", cores=int(workers), kind="oracle",
                sample=(f"{len(cols)} of the {m} columns factorised and solved with SuperLU "
                        f"in a pool of {workers} processes ({wall:.2f} s wall, "
                        f"{np.mean(per):.3f} s per column), scaled to all {m} columns"))


def profiled(L, run_once, steps, torch):
    """Kernel table of `run_once` (which must launch eagerly): one run records
    the algorithmic work per launch, `steps` more the HIP-event times."""
    L.profile_enable(2)
    run_once()
    torch.cuda.synchronize()
    work = L.profile_read()
    L.profile_enable(1)
    for _ in range(steps):
        run_once()
    torch.cuda.synchronize()
    times = L.profile_read()
    L.profile_enable(0)
    return kernel_table(work, times, steps)


def roofline_of(ktab, source):
    """The dominant modelled kernel of a kernel table, as the bench line's
    roofline object (event timing; no counter traffic for this workload)."""
    if not ktab:
        return None
    total = sum(r["ms_per_step"] for r in ktab.values())
    modelled = [(r["ms_per_step"], k) for k, r in ktab.items() if "achieved" in r]
    if not modelled:
        return None
    _, k = max(modelled)
    r = ktab[k]
    return dict(bound=r["bound"], achieved=r["achieved"], peak=r["peak"], unit=r["unit"],
                frac=r["frac"], traffic=None, kernel=k, work_per_launch=r["work_per_launch"],
                time_share=r["ms_per_step"] / total, avg_launch_us=r["avg_launch_us"],
                source=source)


def cpu_oracle_solve(K, d, f, cap, tol, res_tol):
    """Seconds of one oracle solve (median SuperLU solve + FP64 ChebyshevT)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle import chebyshev as och
    from oracle import driver as odrv
    from oracle import lowrank as olr
    m = d.shape[1]
    dbar = och.mean_parameters(d)
    P = och.DirectPreconditioner(och.mean_preconditioner(K, dbar))
    c, dc = och.chebyshev_interval(d, dbar)
    ref = np.linalg.norm(f) * np.sqrt(m)
    t0 = time.perf_counter()
    jmed = odrv.upper_median_offset(m)
    xt = spla.splu(sp.csc_matrix(olr.column_operator(K, d, jmed))).solve(f)
    B = odrv.median_rhs(K, d, f, xt)
    _, info = och.chebyshev_t(K, d, B, P, c, dc, cap, tol, res_tol, ref, max_iter=60)
    return time.perf_counter() - t0, info.iters


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(cfg):
    """The FP64 oracle solving the same problem on the host: median-parameter
    direct solve, then ChebyshevT with SVD truncation to the same tolerance.
    The preconditioner factorisation is set-up (as on the GPU) and not timed."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle import chebyshev as och
    from oracle import driver as odrv
    from oracle import lowrank as olr
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    dbar = och.mean_parameters(d)
    P = och.DirectPreconditioner(och.mean_preconditioner(K, dbar))
    c, dc = och.chebyshev_interval(d, dbar)
    ref = np.linalg.norm(f) * np.sqrt(m)
    t0 = time.perf_counter()
    jmed = odrv.upper_median_offset(m)
    xt = spla.splu(sp.csc_matrix(olr.column_operator(K, d, jmed))).solve(f)
    B = odrv.median_rhs(K, d, f, xt)
    S, info = och.chebyshev_t(K, d, B, P, c, dc, cfg["rank_cap"], cfg["trunc_tol"],
                              cfg["res_tol"], ref, max_iter=40)
    secs = time.perf_counter() - t0
    hi = host_info()
    workers = max(1, min(16, hi["cpus_available"]))
    direct = consecutive_direct(cfg, workers, sample=2 * workers)
    return dict(value=secs, unit="s", cores=int(cores), kind="oracle", host=hi,
                consecutive_direct=direct,
                speedup_lowrank_vs_direct=direct["value"] / secs,
                sample=(f"one complete solve of the same workload (n={K[0].shape[0]}, m={m}): "
                        f"median-parameter SuperLU solve + FP64 ChebyshevT with SVD truncation, "
                        f"{info.iters} iterations to relres {info.history[-1] / ref:.2e} "
                        f"(preconditioner factorisation excluded, as on the GPU; SuperLU "
                        f"single-threaded, BLAS on {cores} threads)"))


def spmm_roofline(L, ops, K, ranks, torch, reps=20):
    """The solver's SpMM on the workload's own operators, alone, at the given
    widths (fp64 and fp32; the autotuned shape; only the operators' non-empty
    rows visited, as inside the solve).  Algorithmic bytes per launch
    as the measurement spec counts them: entries and column indices of every
    operator, row pointers and output rows of the operators' non-empty rows
    only (K_1, K_2 live on the solid box), U read once.  Timed two ways with
    HIP events on the library's stream: warm (back-to-back launches, the
    working set stays in the 256 MiB last-level cache) and cold (a 1 GiB
    buffer is written between launches, so every byte comes from HBM)."""
    n, q = K[0].shape[0], len(K)
    nnz = sum(k.nnz for k in K)
    rows = [int(np.count_nonzero(np.diff(k.indptr))) for k in K]
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
    out = []
    for dt, v, name in ((torch.float64, 8, "f64"), (torch.float32, 4, "f32")):
        for r in ranks:
            ld = max(8, (r + 7) // 8 * 8)
            U = torch.randn((n, ld), dtype=dt, device="cuda")
            W = torch.zeros((q * n, ld), dtype=dt, device="cuda")
            for _ in range(3):
                ops.spmm_dev(U, W, r, skip_empty=True)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                ops.spmm_dev(U, W, r, skip_empty=True)
            e1.record()
            torch.cuda.synchronize()
            t_warm = e0.elapsed_time(e1) / reps * 1e-3
            cold = []
            for _ in range(reps):
                flush.fill_(1.0)
                a0 = torch.cuda.Event(enable_timing=True)
                a1 = torch.cuda.Event(enable_timing=True)
                a0.record()
                ops.spmm_dev(U, W, r, skip_empty=True)
                a1.record()
                torch.cuda.synchronize()
                cold.append(a0.elapsed_time(a1) * 1e-3)
            t = float(np.median(cold))
            b = nnz * (v + 4) + sum(rr + 1 for rr in rows) * 4 + n * r * v + sum(rows) * r * v
            out.append(dict(dtype=name, r=int(r), avg_launch_us=t * 1e6, bytes_per_launch=int(b),
                            achieved=b / t / 1e9, peak=8000.0, unit="GB/s", frac=b / t / 8e12,
                            cache="cold (1 GiB written between launches), median of "
                                  f"{reps}", warm_us=t_warm * 1e6,
                            warm_frac=b / t_warm / 8e12))
    return out


def orthogonality(L, ctx, prob, n, m, torch, r0):
    """max |Q^T Q - I| of the solution's correction factors (after the r0
    columns of the fixed initial term), and of the factors one
    truncation returns at c2's widest concatenation (k = 124 columns: the
    residual [F | K_i S] at rank cap 40) in each precision of its passes.
    The products Q^T Q are formed in fp64 (torch on the device)."""
    U, _, V = prob.solution()
    U, V = U[:, r0:], V[:, r0:]
    sol = dict(U=float(np.abs(U.T @ U - np.eye(U.shape[1])).max()) if U.size else 0.0,
               V=float(np.abs(V.T @ V - np.eye(V.shape[1])).max()) if V.size else 0.0,
               rank=int(U.shape[1]))
    k, cap = 124, 40
    rng = np.random.default_rng(7)
    A = rng.standard_normal((n, k)) * rng.uniform(0.1, 10, k)
    B = rng.standard_normal((m, k))
    c = np.logspace(0, -9, k)
    out = dict(solution=sol)
    for name, tdt, bf16 in (("f64", torch.float64, False), ("f32", torch.float32, False),
                            ("bf16_first_pass", torch.float32, True)):
        Ad = torch.from_numpy(A).to(device="cuda", dtype=tdt)
        Bd = torch.from_numpy(B).to(device="cuda", dtype=tdt)
        Ud = torch.zeros((n, cap), dtype=tdt, device="cuda")
        Vd = torch.zeros((m, cap), dtype=tdt, device="cuda")
        _, r = L.truncate_dev(ctx, Ad, c, Bd, cap, 1e-8, Ud, Vd, bf16=bf16)
        eye = torch.eye(r, dtype=torch.float64, device="cuda")
        u = Ud[:, :r].double()
        v = Vd[:, :r].double()
        out[f"truncation_k{k}_{name}"] = dict(
            U=float((u.T @ u - eye).abs().max()), V=float((v.T @ v - eye).abs().max()), rank=r)
        del Ad, Bd, Ud, Vd, u, v
    torch.cuda.synchronize()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); the "
              f"multi-GPU sharding of the path is described, not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.calibrate_copy:
        # a plain copy of known size: what the HBM byte counters read for it
        # calibrates their readings on the solver's kernels
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)
        return
    from paper_2008_10275_amd import lrcheb as L
    L.load()
    if a.workload == "c3":
        main_batched(a, L, torch)
        return
    if a.workload == "c4":
        main_surrogate(a, L, torch)
        return

    cfg, ctx, ops, prob, setup_s = problem_setup(L, a.workload, a.small)
    opts = solve_opts(L, cfg, a.precision, eager=int(a.eager), recurrence=a.recurrence)
    res_tol = cfg["res_tol"]

    # warm-up (also captures the graphs and tunes the SpMM shapes)
    for _ in range(max(1, a.warmup)):
        one_solve(prob, opts, res_tol)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        infos.append(one_solve(prob, opts, res_tol))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / a.steps * 1e3

    # per-kernel times: the timed steps replay HIP graphs, inside which events
    # cannot bracket single kernels, so the same solve is repeated with every
    # step launched directly (eager) and bracketed by events on the library's
    # stream; the first repeat also records the algorithmic work per launch
    prof_work, prof_time, eager_ms = {}, {}, None
    if not a.no_profile:
        oe = solve_opts(L, cfg, a.precision, eager=1, recurrence=a.recurrence)
        L.profile_enable(2)
        one_solve(prob, oe, res_tol)
        torch.cuda.synchronize()
        prof_work = L.profile_read()
        L.profile_enable(1)
        t2 = time.perf_counter()
        for _ in range(a.steps):
            one_solve(prob, oe, res_tol)
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t2) / a.steps * 1e3
        prof_time = L.profile_read()
        L.profile_enable(0)

    # plain FP64 form of the same solve, for the time-to-tolerance comparison
    fp64 = None
    if a.precision != "fp64" and not a.no_fp64_compare:
        o64 = solve_opts(L, cfg, "fp64")
        one_solve(prob, o64, res_tol)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f_infos = [one_solve(prob, o64, res_tol) for _ in range(a.steps)]
        torch.cuda.synchronize()
        fp64 = dict(seconds=(time.perf_counter() - t1) / a.steps, iters=f_infos[-1]["iters"],
                    relres=f_infos[-1]["relres"], recurrence="direction")
        if a.recurrence != "direction":
            # fp64 in the timed solve's recurrence: what the precision alone buys
            o3 = solve_opts(L, cfg, "fp64", recurrence=a.recurrence)
            one_solve(prob, o3, res_tol)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            g_infos = [one_solve(prob, o3, res_tol) for _ in range(a.steps)]
            torch.cuda.synchronize()
            fp64["same_recurrence"] = dict(seconds=(time.perf_counter() - t2) / a.steps,
                                           iters=g_infos[-1]["iters"],
                                           relres=g_infos[-1]["relres"],
                                           recurrence=a.recurrence)

    # the other mixed form (fp32 ChebyshevT inside fp64 refinement), for reference
    refine = None
    if a.precision == "dir" and not a.no_fp64_compare:
        orf = solve_opts(L, cfg, "mixed", recurrence=a.recurrence)
        one_solve(prob, orf, res_tol)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        r_infos = [one_solve(prob, orf, res_tol) for _ in range(a.steps)]
        torch.cuda.synchronize()
        refine = dict(seconds=(time.perf_counter() - t3) / a.steps, iters=r_infos[-1]["iters"],
                      refinements=r_infos[-1]["refinements"], relres=r_infos[-1]["relres"])

    # the same solve in the other form of the recurrence, for reference
    other = None
    if cfg["ops"].dim == 2 and a.precision != "fp64" and not a.no_fp64_compare:
        oname = "direction" if a.recurrence == "three_term" else "three_term"
        oo = solve_opts(L, cfg, a.precision, recurrence=oname)
        one_solve(prob, oo, res_tol)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        o_infos = [one_solve(prob, oo, res_tol) for _ in range(a.steps)]
        torch.cuda.synchronize()
        other = dict(recurrence=oname, seconds=(time.perf_counter() - t5) / a.steps,
                     iters=o_infos[-1]["iters"], relres=o_infos[-1]["relres"])

    ktab = kernel_table(prof_work, prof_time, a.steps) if prof_time else {}
    roof = None
    if ktab:
        total = sum(r["ms_per_step"] for r in ktab.values())
        modelled = [(r["ms_per_step"], k) for k, r in ktab.items() if "achieved" in r]
        dom_all = max((r["ms_per_step"], k) for k, r in ktab.items())
        if modelled:
            _, k = max(modelled)
            r = ktab[k]
            same = a.workload == "c2" and a.precision == "dir" and not a.small
            rp_us = rocprof_avg_us(k) if same else None
            rp = None
            if rp_us:
                scale = 1e9 if r["unit"] == "GB/s" else 1e12
                ach = r["work_per_launch"] / (rp_us * 1e-6) / scale
                rp = dict(avg_launch_us=rp_us, achieved=ach, frac=ach / r["peak"],
                          source="profiles/solve_dir_c2_kernels.md (rocprofv3 kernel trace)")
            roof = dict(bound=r["bound"], achieved=r["achieved"], peak=r["peak"], unit=r["unit"],
                        frac=r["frac"], traffic=measured_traffic(k) if same else None, kernel=k,
                        rocprof=rp,
                        work_per_launch=r["work_per_launch"],
                        time_share=r["ms_per_step"] / total,
                        avg_launch_us=r["avg_launch_us"],
                        source=("HIP events on the library stream around every launch, in a "
                                "repeat of the timed steps with eager launches"))
            if dom_all[1] != k:
                roof["dominant_unmodelled"] = dict(kernel=dom_all[1],
                                                   time_share=dom_all[0] / total)

    cpu = None
    if not a.no_cpu and cfg["ops"].dim == 2:
        # (3D: SuperLU's fill on the 27-point pattern puts one column solve
        # beyond the host budget; the 2D line carries the host baseline)
        cpu = cpu_baseline(cfg)

    # the 3D workload: every precision form of the same solve
    forms = None
    if cfg["ops"].dim == 3 and not a.no_fp64_compare:
        forms = {}
        for pname in ("fp64", "dir", "mixed", "bf16gram"):
            of = solve_opts(L, cfg, pname,
                            recurrence="direction" if pname == "fp64" else a.recurrence)
            one_solve(prob, of, res_tol)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            fi = [one_solve(prob, of, res_tol) for _ in range(a.steps)]
            torch.cuda.synchronize()
            forms[pname] = dict(ms=(time.perf_counter() - t4) / a.steps * 1e3,
                                iters=fi[-1]["iters"], refinements=fi[-1]["refinements"],
                                rank=fi[-1]["rank"], relres=fi[-1]["relres"])

    last = infos[-1]
    # the SpMM alone at the solution's rank and at the rank cap
    spmm = None if a.no_spmm_roofline else spmm_roofline(
        L, ops, cfg["ops"].K, sorted({max(1, int(last["rank"])), int(cfg["rank_cap"])}), torch)
    n, m = cfg["ops"].K[0].shape[0], cfg["d"].shape[1]
    orth = None if a.no_orthogonality else orthogonality(L, ctx, prob, n, m, torch,
                                                         int(last.get("rank_x0", 0)))
    line = {
        "metric": "time to rel. residual 1e-6 (s)" if res_tol == 1e-6 else
                  f"time to rel. residual {res_tol:g} (s)",
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "bf16gram": "bf16+f32+f64"}.get(a.precision, "f32+f64"),
        "data": "synthetic",
        "config": {"workload": workload_name(cfg, n, m), "n": int(n), "m": int(m),
                   "q": len(cfg["ops"].K),
                   "rank_cap": cfg["rank_cap"], "trunc_tol": cfg["trunc_tol"],
                   "res_tol": res_tol,
                   "recurrence": a.recurrence,
                   "precision": {"mixed": "fp32 inner ChebyshevT, fp64 residual + refinement",
                                 "dir": ("fp64 iterate and residual, fp32 preconditioner "
                                         "solves and direction updates"),
                                 "fp64": "fp64",
                                 "bf16gram": ("fp32 inner ChebyshevT with bf16 first-pass "
                                              "Gram products, fp64 residual + refinement")
                                 }[a.precision]},
        "result": {"relres_fp64": last["relres"], "max_col_relres": last["max_col_relres"],
                   "iters": last["iters"], "refinements": last["refinements"],
                   "rank": last["rank"], "median_iters": last["median_iters"],
                   "setup_s": setup_s},
        "eager_ms_per_step": eager_ms,
        "fp64_plain": fp64,
        "mixed_refinement": refine,
        "other_recurrence": other,
        "orthogonality": orth,
        "forms": forms,
        "speedup_vs_fp64": (fp64["seconds"] / (ms / 1e3)) if fp64 else None,
        "roofline": roof,
        "spmm_roofline": spmm,
        "kernels": ktab,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
