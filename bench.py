"""Benchmark: space-time DOF x V-cycles per second on one GPU.

Workload: 2D linear reaction-diffusion u_t = nu Lap u - lambda u, nu = 1e-2,
lambda = 1, periodic [0,1]^2, 256 x 256 points, M = 3 right Radau nodes,
N = 256 steps, T = 1 (50,331,648 space-time unknowns), seeded random
Fourier initial data.  One step = one FP64 solve from a zero initial guess
to a relative residual of 1e-12.  Also reported: time to a 1e-10 residual
in FP64 and in mixed precision; the longest kernel of the V-cycle and the
whole V-cycle against the HBM roofline (HIP events on the solver's stream,
algorithmic bytes from the level shapes); the other synthetic workloads
with their errors against the CPU oracle; and the oracle itself (the
sequential Radau IIA stepper with a sparse direct solve per step) timed on
the host.

Prints one JSON line.  Only N = 1 GPU is supported.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the V-cycle's longest kernels from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs, scaled by what the counters read for a device copy of known
# size (FETCH x 2, WRITE x 1; profiles/k_prolong_smooth_blk_rd2d_level0.md),
# valid only while the kernel's source files (one hash over their
# concatenation) are the ones the counters were taken on.
TRAFFIC = {
    "k_prolong_smooth_blk": {"sources": ["kernels_impl.hpp", "launchers.hpp"],
                             "sha256_prefix": "e684e6ec938869c4",
                             "bytes_per_launch": 531.6e6 + 402.7e6},
    # the fused level-0 sweep + restriction and its run-boundary pass
    # (profiles/k_smooth_restrict_rd2d_level0.md)
    "k_smooth_restrict": {"sources": ["smooth_restrict.hip", "kernels_impl.hpp"],
                          "sha256_prefix": "4ecd665be0ad03a9",
                          "bytes_per_launch": 424.8e6 + 607.7e6 + 18.4e6 + 13.8e6},
}


def sources_hash(files):
    """sha256 prefix (16 hex digits) of the concatenated kernel sources."""
    import hashlib
    d = b"".join(open(os.path.join(ROOT, "paper_2006_12883_amd", "csrc", f), "rb").read() for f in files)
    return hashlib.sha256(d).hexdigest()[:16]


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch of `kernel`, while its source
    files hash to the ones the counters were taken on (else None)."""
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    return t["bytes_per_launch"] if sources_hash(t["sources"]) == t["sha256_prefix"] else None


def sr_run_len(nx, ny, N, chunk=16):
    """Slabs per workgroup of the fused level-0 sweep + restriction, as its
    launcher chooses them: whole smoother chunks, doubled while the launch
    keeps at least 512 workgroups (tiles of 64 x 16 fine points)."""
    tiles = (nx // 64) * (ny // 16)
    rl = chunk
    while rl < N and tiles * (-(-N // (2 * rl))) >= 512:
        rl *= 2
    return rl


def sr_bytes(l0, l1, word=8, chunk=16, cs=4, zs=True):
    """Algorithmic bytes of the fused level-0 sweep + restriction with its
    run-boundary pass: U in, U' out, f_c (and the coarse first sweep U_c) out,
    one plane of cout . d per run boundary out; then per boundary that plane
    in, f_c of one coarse slab and U_c of one coarse chunk read and written."""
    P, Pc = l0["nx"] * l0["ny"], l1["nx"] * l1["ny"]
    dof0, c = P * l0["N"] * l0["M"], Pc * l1["N"] * l1["M"]
    nb = -(-l0["N"] // sr_run_len(l0["nx"], l0["ny"], l0["N"], chunk)) - 1
    kern = 2 * word * dof0 + word * c * (2 if zs else 1) + word * P * nb
    fix = nb * (word * P + 2 * word * l0["M"] * Pc * (1 + (cs if zs else 0)))
    return float(kern + fix)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (Allen-Cahn Newton, adjoint, batch)")
    ap.add_argument("--kernel-iters", type=int, default=20)
    ap.add_argument("--only", choices=EXTRA_GROUPS, default=None,
                    help="run only this group of the other workloads and print their JSON (for traces)")
    ap.add_argument("--krylov-only", action="store_true",
                    help="only the flexible GMRES lines on the 256^2 workload (used for the Krylov "
                         "kernel trace)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only time the level-0 kernels and a plain device copy of the "
                         "same bytes (used for the HBM counter runs)")
    ap.add_argument("--cycle-only", action="store_true",
                    help="only time back-to-back V-cycles (used for the kernel traces)")
    return ap.parse_args()


def cycle_bytes(levels, word=8, fused0=False):
    """Algorithmic HBM bytes of one V(1,1) cycle with the fused kernels, from
    the level shapes (levels[l] = dict(nx, ny, N, M, kind)):
      level 0: pre-smoothing reads U, writes U' (the right-hand side is
        generated from u0); the restriction reads U and writes f_c and the
        coarse level's first sweep U_c (fused0: the two as one kernel, see
        sr_bytes); the prolongation + post-smoothing reads U and e_c and
        writes U';
      levels 0 < l < coarsest: the restriction reads U and f, writes f_c (and
        U_c unless the next level is the coarsest); the prolongation +
        post-smoothing reads U, f, e_c and writes U';
      coarsest: the exact solve reads f and writes U.
    Returns (bytes, [bytes per level])."""
    dof = [lv["nx"] * lv["ny"] * lv["N"] * lv["M"] for lv in levels]
    L = len(levels) - 1
    per = []
    for l in range(L + 1):
        if l == L:
            per.append(2 * word * dof[l])
            break
        c = dof[l + 1]
        b = 0
        if l == 0:
            if fused0:
                b += sr_bytes(levels[0], levels[1], word, zs=L > 1)  # sweep + restriction
            else:
                b += 2 * word * dof[0]                 # pre-smoothing
                b += word * dof[0] + 2 * word * c      # restriction + coarse first sweep
            b += 2 * word * dof[0] + word * c      # prolongation + post-smoothing
        else:
            b += 2 * word * dof[l] + word * c * (2 if l + 1 < L else 1)
            b += 3 * word * dof[l] + word * c
        per.append(b)
    return float(sum(per)), [float(x) for x in per]


def model_cycle_bytes(levels, nu_pre=1, nu_post=1, word=8):
    """Bytes of one V-cycle under the unfused per-unit word counts of the
    method (every sweep reads U and b and writes U: 3 words; residual +
    restriction 2 + 1/c words; prolongation + correction 2 + 1/c words, c the
    coarsening factor of the step; the coarsest exact solve reads f and writes
    U), summed over the levels: the bytes the V-cycle moves without fusion."""
    dof = [lv["nx"] * lv["ny"] * lv["N"] * lv["M"] for lv in levels]
    total = 0.0
    for l in range(len(levels)):
        if l == len(levels) - 1:
            total += 2 * word * dof[l]
            break
        c = dof[l] / dof[l + 1]
        total += word * dof[l] * (3 * (nu_pre + nu_post) + 4 + 2 / c)
    return total


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)",
                             "CPU max MHz"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    return info


def cpu_baseline(prob, u0, gpu_solutions, gpu_seconds_per_solve):
    """The CPU leg: the oracle's sequential Radau IIA stepper (collocation
    form, one sparse LU of the stage matrix I - dt Q (x) L, then one
    triangular solve pair per step) on one host thread, timed on a bounded
    sample: the factorization and the first `steps` steps; the full solve
    time is the factorization plus N times the per-step time.  Secondary: the
    oracle's NumPy V-cycle rate on the same workload.  The oracle's Fourier
    closed form of the workload gives the error of each GPU result."""
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits
    from oracle import fourier, mg, radau, space, stepper
    steps = 8
    with threadpool_limits(limits=1):
        Q = radau.tables(prob["M"])["Q"]
        L = space.linear_operator(prob)
        t0 = time.perf_counter()
        S = stepper._stage_matrix(Q, L, prob["dt"])
        lu = spla.splu(S)
        t_factor = time.perf_counter() - t0
        u = np.asarray(u0, dtype=np.float64).reshape(-1)
        t1 = time.perf_counter()
        for _ in range(steps):
            Un = lu.solve(np.tile(u, prob["M"]))
            u = Un[(prob["M"] - 1) * u.size:]
        t_step = (time.perf_counter() - t1) / steps
        del lu, S
        levels, kinds = mg.hierarchy(prob)
        f = mg.rhs(levels, u0)
        U = np.zeros(levels[0].shape)
        ncyc = 2
        t2 = time.perf_counter()
        for _ in range(ncyc):
            U = mg.vcycle(levels, kinds, U, f)
        t_cyc = (time.perf_counter() - t2) / ncyc
        del U, f
        t3 = time.perf_counter()
        ref = fourier.solve_linear_periodic(prob, u0)
        tf = time.perf_counter() - t3
    dof = float(np.prod(levels[0].shape))
    t_solve = t_factor + prob["N"] * t_step
    errs = {}
    for k, V in gpu_solutions.items():
        errs[k] = {"rel_err": float(np.linalg.norm(V - ref) / np.linalg.norm(ref)),
                   "rel_err_at_T": float(np.linalg.norm(V[-1, -1] - ref[-1, -1]) / np.linalg.norm(ref[-1, -1]))}
    return {"value": t_solve, "unit": "s per full solve (time to solution of the 256^2 x 3 x 256 workload)",
            "cores": 1, "kind": "oracle",
            "sample": "sequential Radau IIA stepper (scipy splu of the 196,608-unknown stage matrix, then "
                      "%d of the %d steps), 1 thread; full solve = factorization + %d x per-step time; "
                      "%.1f s of CPU work" % (steps, prob["N"], prob["N"], t_factor + steps * t_step),
            "factor_seconds": t_factor, "seconds_per_step": t_step,
            "gpu_seconds_per_solve_to_1e-12": gpu_seconds_per_solve,
            "host": host_info(),
            "mg_vcycle": {"value": dof / t_cyc, "unit": "DOF*V-cycles/s", "seconds_per_vcycle": t_cyc,
                          "sample": "%d consecutive V-cycles of the oracle's NumPy multigrid (oracle.mg) on "
                                    "the full workload from a zero guess, 1 thread" % ncyc},
            "fourier_closed_form_seconds": tf,
            "gpu_error_vs_oracle": errs}


def _events(stream, iters, fn):
    """Average milliseconds of fn() over iters launches, HIP events on `stream`."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(stream)
    for _ in range(iters):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / iters


def time_kernels(h, U, u0, iters):
    """The level-0 kernels of the V-cycle through their component entry points
    (smoothing sweep, residual restriction, fused prolongation + smoothing),
    back-to-back V-cycles, and a plain copy of the smoother's byte count, each
    timed with HIP events on the solver's stream."""
    import ctypes
    import torch
    from paper_2006_12883_amd import binding as B
    lv = h.levels()
    c = lv[1]
    shape1 = (c["N"], c["M"], c["ny"], c["nx"])
    Uin = U.clone()
    Uout = torch.empty_like(U)
    ec = torch.randn(shape1, dtype=torch.float64, device=U.device)
    fc = torch.empty(shape1, dtype=torch.float64, device=U.device)
    s = h.stream
    dof0 = float(U.numel())
    dof1 = float(ec.numel())
    k = {}
    k["k_smooth_blk"] = (_events(s, iters, lambda: h.smooth(0, Uin, Uout, u0=u0)), 16.0 * dof0)
    k["k_restrict_blk"] = (_events(s, iters, lambda: h.restrict_residual(0, Uin, fc, u0=u0)), 8.0 * dof0 + 8.0 * dof1)
    k["k_prolong_smooth_blk"] = (_events(s, iters, lambda: h.prolong_smooth(0, ec, Uout, Uin=Uin, u0=u0)),
                                 16.0 * dof0 + 8.0 * dof1)
    # the V-cycle's level-0 sweep and restriction as one kernel, where the grid allows it
    uc = torch.empty(shape1, dtype=torch.float64, device=U.device)
    try:
        h.smooth_restrict(0, Uout, fc, Uin=Uin, uc=uc, u0=u0)
        fused0 = True
    except B.STMGError:
        fused0 = False
    if fused0:
        k["k_smooth_restrict"] = (_events(s, iters, lambda: h.smooth_restrict(0, Uout, fc, Uin=Uin, uc=uc, u0=u0)),
                                  sr_bytes(lv[0], lv[1], zs=True))
    kernels = {name: {"ms": ms, "bytes": b, "GBs": b / (ms * 1e-3) / 1e9,
                      "in_cycle": name == "k_prolong_smooth_blk" or (name == "k_smooth_restrict") == fused0}
               for name, (ms, b) in k.items()}
    # whole cycles, no host synchronization in between
    V = torch.zeros_like(U)
    L = B.lib()
    cyc = lambda: B.check(L.stmg_vcycle(h.h, ctypes.c_void_p(u0.data_ptr()), ctypes.c_void_p(V.data_ptr()), None),
                          "stmg_vcycle")
    cyc_ms = _events(s, iters, cyc)
    x = torch.ones(U.numel(), dtype=torch.float64, device=U.device)
    y = torch.empty_like(x)
    with torch.cuda.stream(s):
        c_ms = _events(s, iters, lambda: y.copy_(x))
    del Uin, Uout, ec, fc, uc, V, x, y
    return kernels, cyc_ms, lv, c_ms, 2.0 * U.numel() * 8, fused0


EXTRA_GROUPS = ("heat1d", "allen_cahn", "adjoint", "batch", "sdc", "pfasst", "hierarchies", "krylov", "paper")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def extras(dev, only=None):
    """The other synthetic workloads, each timed once after a warm-up call
    (only: one of EXTRA_GROUPS, else all)."""
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    out = {}
    if only in (None, "heat1d"):
        out.update(_extra_heat1d(dev))
    if only in (None, "allen_cahn"):
        out.update(_extra_allen_cahn(dev))
    if only in (None, "adjoint"):
        out.update(_extra_adjoint(dev))
    if only in (None, "batch"):
        out.update(_extra_batch(dev))
    if only in (None, "sdc"):
        out.update(_extra_sdc(dev))
    if only in (None, "pfasst"):
        out.update(_extra_pfasst(dev))
    if only in (None, "hierarchies"):
        out.update(_extra_hierarchies(dev))
    if only in (None, "krylov"):
        out["krylov_rd2d_fp64_to_1e-10"] = krylov_lines(dev)
        print("krylov done", file=sys.stderr, flush=True)
    if only in (None, "paper"):
        out["paper_examples_1d"] = paper_examples(dev)
        print("paper examples done", file=sys.stderr, flush=True)
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _extra_heat1d(dev):
    """The 1D heat workload (64 points, M = 2, N = 16, 2,048 unknowns), FP64 to
    1e-12: cache-resident and latency-bound, so only its absolute time; the
    error is against the oracle's stepper."""
    import torch
    import stmg_inputs as si
    from oracle import stepper
    from paper_2006_12883_amd import stmg
    prob = si.config("heat1d")
    u0n = si.initial("heat1d", prob)
    u0 = torch.as_tensor(u0n).to(dev)
    h = stmg.Handle(prob, device=dev)
    U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
    times = []
    for _ in range(6):
        U.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = h.solve(u0, U)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ref = stepper.solve_linear(prob, u0n)
    V = U.cpu().numpy()
    print("heat1d done", file=sys.stderr, flush=True)
    return {"heat1d_64_M2_N16_fp64_to_1e-12": {
        "ms_median": 1e3 * float(np.median(times[1:])), "vcycles": st["cycles"], "rel_res": st["rel_res"],
        "levels": len(h.levels()), "rel_err_vs_oracle": _rel(V, ref), "rel_err_at_T": _rel(V[-1, -1], ref[-1, -1])}}


def _extra_allen_cahn(dev):
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    out = {}
    # 2D Allen-Cahn 512^2 x M=3 x N=512 by Newton: FP32 V-cycles inside FP64
    # refinement, and all-FP64 cycles, to the same Newton tolerance; errors
    # against the stored oracle solution (tests/golden/make_ac2d_golden.py)
    prob = si.config("ac2d")
    u0 = torch.as_tensor(si.initial("ac2d", prob)).to(dev)
    gpath = os.path.join(GOLDEN, "ac2d_512_golden.npz")
    g = np.load(gpath) if os.path.exists(gpath) else None
    dof = float(prob["N"] * prob["M"] * 512 * 512)
    for prec in ("mixed", "fp64"):
        h = stmg.Handle(prob, device=dev, precision=prec, newton_rtol=1e-10)
        U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
        h.solve(u0, U)
        U.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = h.solve(u0, U)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        line = {"seconds_to_1e-10": t, "newton_its": st["newton_its"], "vcycles": st["cycles"],
                "refinements": st["refinements"], "rel_res": st["rel_res"], "dof": int(dof),
                "dof_vcycles_per_s": dof * st["cycles"] / t}
        if g is not None:
            line["rel_err_vs_oracle_at_T"] = _rel(U[-1, -1].cpu().numpy(), g["uT"])
            line["rel_err_vs_oracle_at_T_half"] = _rel(U[prob["N"] // 2 - 1, -1].cpu().numpy(), g["umid"])
            norms = torch.linalg.vector_norm(U.reshape(prob["N"], prob["M"], -1), dim=2).cpu().numpy()
            line["max_rel_err_slab_norms"] = float(np.abs(norms / g["norms"] - 1).max())
        out["allen_cahn_512x512_M3_N512_" + prec] = line
        del h, U
        torch.cuda.empty_cache()
    if g is not None:
        out["allen_cahn_oracle"] = {"seconds": float(g["seconds"]), "factorizations": int(g["factors"]),
                                    "newton_its": int(g["newton_its"]),
                                    "where": "build container host, 1 core (stored with the golden)"}
    print("allen-cahn done", file=sys.stderr, flush=True)
    return out


def _extra_adjoint(dev):
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    out = {}
    # adjoint on the 256^2 workload: gradient w.r.t. u0 and nu, FP64 and mixed
    # precision (FP32 cycles on the transposed system inside FP64 refinement)
    # to the same tolerance; errors against the stored oracle gradients
    # (tests/golden/make_adj2d_golden.py)
    prob = si.config("adj2d")
    u0n = si.initial("adj2d", prob)
    u0 = torch.as_tensor(u0n).to(dev)
    tgt = torch.as_tensor(si.u_tgt_adj2d(prob)).to(dev)
    gpath = os.path.join(GOLDEN, "adj2d_256_golden.npz")
    gold = np.load(gpath) if os.path.exists(gpath) else None
    for prec in ("fp64", "mixed"):
        h = stmg.Handle(prob, device=dev, precision=prec, rtol=1e-11)
        U, _ = h.solve(u0)
        g = 2.0 * (U[-1, -1] - tgt)
        h.adjoint(U, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gu0, gnu, st = h.adjoint(U, g)
        torch.cuda.synchronize()
        line = {"seconds": time.perf_counter() - t0, "vcycles": st["cycles"], "rel_res": st["rel_res"],
                "dL_dnu": gnu}
        if gold is not None:
            line["rel_err_grad_u0_vs_oracle"] = _rel(gu0.cpu().numpy(), gold["grad_u0"])
            line["rel_err_dL_dnu_vs_oracle"] = abs(gnu / float(gold["grad_nu"]) - 1.0)
        out["adjoint_256x256_M3_N256_" + prec + "_to_1e-11"] = line
        del h, U
        torch.cuda.empty_cache()
    print("adjoint done", file=sys.stderr, flush=True)
    return out


def _extra_batch(dev):
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    out = {}
    # 64 batched problems, FP32 V-cycles in FP64 refinement to 1e-10
    probs = si.batch64()
    u0s = [torch.as_tensor(si.batch_u0(p, i)).to(dev) for i, p in enumerate(probs)]
    # launch shapes from the batch autotuner (cached in $STMG_TUNE_CACHE, else
    # a file under /tmp); setup, tuning included, is outside the timed solve
    os.environ.setdefault("STMG_TUNE_CACHE", os.path.join("/tmp", "stmg_tune_cache.json"))
    t_setup = time.perf_counter()
    b = stmg.Batch(probs, device=dev, rtol=1e-10, autotune=1)
    t_setup = time.perf_counter() - t_setup
    Us, _ = b.solve(u0s)
    for U in Us:
        U.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Us, sts = b.solve(u0s, Us)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    dofs = [float(np.prod(U.shape)) for U in Us]
    out["batch64_mixed"] = {"seconds_to_1e-10": t, "setup_seconds_with_autotune": t_setup,
                            "autotuned": True, "problems": len(probs), "total_dof": int(sum(dofs)),
                            "max_cycles": max(st["cycles"] for st in sts),
                            "dof_vcycles_per_s": sum(d * st["cycles"] for d, st in zip(dofs, sts)) / t,
                            "max_rel_res": max(st["rel_res"] for st in sts)}
    del b, Us
    torch.cuda.empty_cache()
    out["batch64_mixed"]["cpu_baseline"] = _batch_cpu_baseline(probs, t)
    print("batch done", file=sys.stderr, flush=True)
    return out


def _batch_cpu_baseline(probs, gpu_seconds):
    """The oracle's Fourier closed form (oracle.fourier, the exact collocation
    solution of a periodic linear problem) on a bounded sample of the batch:
    every 4th problem, over a pool of threads, one per host core up to 16
    (numpy's transforms and solves release the interpreter lock for part of
    the work); the time for all 64 problems is extrapolated by unknowns."""
    from concurrent.futures import ThreadPoolExecutor
    import stmg_inputs as si
    from oracle import fourier
    idx = list(range(0, len(probs), 4))
    work = [(probs[i], si.batch_u0(probs[i], i)) for i in idx]
    nthreads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))

    def one(a):
        prob, u0 = a
        return float(np.abs(fourier.solve_linear_periodic(prob, u0)[-1, -1]).max())

    t0 = time.perf_counter()
    with ThreadPoolExecutor(nthreads) as ex:
        list(ex.map(one, work))
    t = time.perf_counter() - t0
    dof = lambda p: p["nx"][0] * p["nx"][1] * p["M"] * p["N"]
    ds = float(sum(dof(p) for p, _ in work))
    da = float(sum(dof(p) for p in probs))
    return {"value": t * da / ds, "unit": "s for the 64 problems (extrapolated by unknowns)", "cores": nthreads,
            "kind": "oracle", "sample": "%d of the %d problems (every 4th), the Fourier closed form, %d threads; "
                                       "%.1f s wall" % (len(work), len(probs), nthreads, t),
            "sample_seconds": t, "sample_dof": ds, "gpu_seconds_to_1e-10": gpu_seconds}


def _extra_sdc(dev):
    """SDC sweeps (the implicit-Euler preconditioned Richardson iteration on the
    collocation form, all slabs at once) on the 256^2 workload: time per sweep
    and the DG residual after each block of sweeps."""
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    prob = si.config("rd2d")
    u0 = torch.as_tensor(si.initial("rd2d", prob)).to(dev)
    h = stmg.Handle(prob, device=dev, sdc=1)
    U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
    h.sdc_sweep(u0, U, 1)
    U.zero_()
    torch.cuda.synchronize()
    rels = []
    t0 = time.perf_counter()
    for _ in range(4):
        rels.append(h.sdc_sweep(u0, U, 4))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    del h, U
    torch.cuda.empty_cache()
    print("sdc done", file=sys.stderr, flush=True)
    return {"sdc_rd2d_fp64": {"sweeps": 16, "seconds_per_sweep": t / 16, "rel_res_after_4_8_12_16": rels}}


def _extra_pfasst(dev):
    """PFASST^L_1 (Sec. 5.2: one sweep per level, M = 1 and bisection in space
    on the coarse levels) beside the multigrid solve, FP64 to 1e-10, on the
    256^2 workload and the 1D heat workload: iterations, time, and the
    difference between the two solutions; inner solves to rtol, or cut to 1 or
    2 V-cycles (pfasst_inner_cycles)."""
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    out = {}
    for cfg in ("rd2d", "heat1d"):
        prob = si.config(cfg)
        u0 = torch.as_tensor(si.initial(cfg, prob)).to(dev)
        h = stmg.Handle(prob, device=dev, rtol=1e-10, max_cycles=200)
        Ur = torch.zeros(h.shape, dtype=torch.float64, device=dev)
        h.solve(u0, Ur, check=False)
        Ur.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, sr = h.solve(u0, Ur, check=False)
        torch.cuda.synchronize()
        line = {"stmg": {"seconds": time.perf_counter() - t0, "vcycles": sr["cycles"], "rel_res": sr["rel_res"]}}
        del h
        for L, inner in ((2, 0), (3, 0), (2, 1), (2, 2), (3, 1)):
            h = stmg.Handle(prob, device=dev, pfasst_levels=L, pfasst_inner_cycles=inner, rtol=1e-10,
                            max_cycles=300)
            U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
            h.pfasst(u0, U, check=False)
            U.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = h.pfasst(u0, U, check=False)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            line["pfasst_L%d" % L + ("_inner%d" % inner if inner else "")] = {"seconds": t, "iterations": st["cycles"], "status": st["status"],
                                      "rel_res": st["rel_res"],
                                      "rel_diff_vs_stmg": float(torch.linalg.norm(U - Ur) / torch.linalg.norm(Ur)),
                                      "seconds_per_iteration": t / max(1, st["cycles"])}
            del h, U
            torch.cuda.empty_cache()
        out["pfasst_%s_fp64_to_1e-10" % cfg] = line
        del Ur
        torch.cuda.empty_cache()
    # Allen-Cahn (512^2 x 3 x 512): IMEX PFASST on 4 levels (the 64^2
    # coarsest level swept slab after slab by Fourier solves) beside Newton
    # around the multigrid solve, FP64 to 1e-10
    prob = si.config("ac2d")
    u0 = torch.as_tensor(si.initial("ac2d", prob)).to(dev)
    h = stmg.Handle(prob, device=dev, rtol=1e-10, newton_rtol=1e-10, max_cycles=200)
    Ur = torch.zeros(h.shape, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sr = h.solve(u0, Ur, check=False)
    torch.cuda.synchronize()
    line = {"stmg_newton": {"seconds": time.perf_counter() - t0, "vcycles": sr["cycles"],
                            "newton_its": sr["newton_its"], "rel_res": sr["rel_res"]}}
    del h
    torch.cuda.empty_cache()
    for inner in (1, 2):
        h = stmg.Handle(prob, device=dev, pfasst_levels=4, pfasst_inner_cycles=inner, rtol=1e-10, max_cycles=300)
        U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = h.pfasst(u0, U, check=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        line["pfasst_imex_L4_inner%d" % inner] = {
            "seconds": t, "iterations": st["cycles"], "status": st["status"], "rel_res": st["rel_res"],
            "rel_diff_vs_stmg": float(torch.linalg.norm(U - Ur) / torch.linalg.norm(Ur)),
            "seconds_per_iteration": t / max(1, st["cycles"])}
        del h, U
        torch.cuda.empty_cache()
    out["pfasst_ac2d_fp64_to_1e-10"] = line
    del Ur
    torch.cuda.empty_cache()
    print("pfasst done", file=sys.stderr, flush=True)
    return out


def _extra_hierarchies(dev):
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    out = {}
    # the paper's three hierarchies (Sec. 5.2) on the 256^2 workload, FP64 to
    # 1e-10: SMG (space only), STMG (space and time at once), SMMG (space and
    # nodes); AUTO semi-coarsening is the headline solve.  SMG also with
    # Galerkin coarse levels R A P (Sec. 4.2), on the default hierarchy and on
    # one run down to the smallest coarse grid, each beside the rediscretized
    # one.
    prob = si.config("rd2d")
    u0 = torch.as_tensor(si.initial("rd2d", prob)).to(dev)
    dof = float(prob["N"] * prob["M"] * 256 * 256)
    variants = {}
    runs = [("auto", {}), ("space", {}), ("spacetime", {}), ("smmg", {}),
            ("space_galerkin", dict(coarse_op="galerkin")),
            ("space_deep", dict(fft_coarse=0)),
            ("space_galerkin_deep", dict(fft_coarse=0, coarse_op="galerkin"))]
    for name, extra in runs:
        h = stmg.Handle(prob, device=dev, coarsen=name.split("_")[0], rtol=1e-10, max_cycles=100, **extra)
        U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
        h.solve(u0, U, check=False)
        U.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = h.solve(u0, U, check=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        lv = h.levels()
        variants[name] = {"seconds": t, "status": st["status"], "vcycles": st["cycles"],
                          "rel_res": st["rel_res"], "levels": len(lv),
                          "coarsest": [lv[-1]["nx"], lv[-1]["ny"], lv[-1]["N"], lv[-1]["M"]],
                          "dof_vcycles_per_s": dof * st["cycles"] / t}
        del h, U
        torch.cuda.empty_cache()
    out["hierarchies_rd2d_fp64_to_1e-10"] = variants
    print("hierarchies done", file=sys.stderr, flush=True)
    return out


def krylov_lines(dev):
    """Flexible GMRES around the AUTO V-cycle on the 256^2 workload, FP64 to
    1e-10, restart 5 and 10, beside the plain iteration."""
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    prob = si.config("rd2d")
    u0 = torch.as_tensor(si.initial("rd2d", prob)).to(dev)
    kry = {}
    for m in (0, 5, 10):
        h = stmg.Handle(prob, device=dev, krylov=m, rtol=1e-10)
        U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
        _, st, t = _timed_solve(h, u0, U)
        kry["plain" if m == 0 else "fgmres%d" % m] = {"seconds": t, "status": st["status"],
                                                      "vcycles": st["cycles"], "rel_res": st["rel_res"]}
        del h, U
        torch.cuda.empty_cache()
    return kry


def _timed_solve(h, u0, U):
    import torch
    h.solve(u0, U, check=False)
    U.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = h.solve(u0, U, check=False)
    torch.cuda.synchronize()
    return U, st, time.perf_counter() - t0


def _timed_pfasst(h, u0, U):
    import torch
    h.pfasst(u0, U, check=False)
    U.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = h.pfasst(u0, U, check=False)
    torch.cuda.synchronize()
    return U, st, time.perf_counter() - t0


def paper_examples(dev):
    """The paper's 1D examples (Sec. 5) on one GPU: the heat example with
    N_x = 1024 and N_t per M from its tables, stopped at 1e-9, with the
    paper's hierarchies (SMG and SMMG 7 levels, STMG 5 levels), plain cycles
    and flexible GMRES around them (true-residual stop), and left-
    preconditioned GMRES (preconditioned-residual stop, as the paper counts);
    and the monodomain example (X = 10,
    T = 2, gamma = 5) with Newton around SMG.  Iteration counts and times are
    context: the paper smooths with ILU(0)-preconditioned GMRES on CPU cores."""
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg
    heat = {}
    runs = [("SMG7_V11", "space", 7, 0, 1), ("SMG7_V11_fgmres10", "space", 7, 10, 1),
            ("SMG7_V33", "space", 7, 0, 3), ("SMG7_V33_fgmres10", "space", 7, 10, 3),
            ("SMG7_V33_leftgmres10", "space", 7, -10, 3),
            ("SMMG7_V33_fgmres30", "smmg", 7, 30, 3), ("STMG5_V33_fgmres30", "spacetime", 5, 30, 3)]
    for M in (1, 2, 3, 4, 5):
        prob = si.paper_heat1d(M)
        u0 = torch.as_tensor(si.u0_paper_heat1d(prob)).to(dev)
        row = {}
        for name, coarsen, levels, m, nu in runs:
            if coarsen == "smmg" and M == 1:
                continue
            h = stmg.Handle(prob, device=dev, coarsen=coarsen, max_levels=levels, krylov=abs(m),
                            krylov_left=1 if m < 0 else 0, nu_pre=nu, nu_post=nu, rtol=1e-9, max_cycles=300)
            U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
            _, st, t = _timed_solve(h, u0, U)
            row[name] = {"ms": 1e3 * t, "status": st["status"], "vcycles": st["cycles"],
                         "rel_res": st["rel_res"]}
            del h, U
        heat["M%d_Nt%d" % (M, prob["N"])] = row
    weak = {}
    for M in (1, 2, 3, 4, 5):
        for Nt, L in si.PAPER_WEAK[M]:
            prob = si.paper_heat1d(M, Nt=Nt)
            u0 = torch.as_tensor(si.u0_paper_heat1d(prob)).to(dev)
            h = stmg.Handle(prob, device=dev, coarsen="space", max_levels=L, krylov=10, nu_pre=3, nu_post=3,
                            rtol=1e-9, max_cycles=300)
            U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
            _, st, t = _timed_solve(h, u0, U)
            weak["M%d_Nt%d_L%d" % (M, Nt, L)] = {"ms": 1e3 * t, "status": st["status"], "vcycles": st["cycles"],
                                                "rel_res": st["rel_res"]}
            del h, U
    mono = {}
    for M in (1, 2, 3, 4, 5):
        prob = si.paper_monodomain(M)
        u0 = torch.as_tensor(si.u0_paper_monodomain(prob)).to(dev)
        h = stmg.Handle(prob, device=dev, coarsen="space", max_levels=7, krylov=10, nu_pre=3, nu_post=3,
                        newton_rtol=1e-9, max_cycles=2000)
        U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
        _, st, t = _timed_solve(h, u0, U)
        mono["M%d_Nt%d" % (M, prob["N"])] = {"ms": 1e3 * t, "status": st["status"], "newton_its": st["newton_its"],
                                            "vcycles": st["cycles"], "rel_res": st["rel_res"]}
        del h, U
    # PFASST^3_1 (Sec. 5.2: M = 1 and bisection on the coarse levels, one sweep
    # per level) on both examples, every slab at once (one slab per core in
    # the paper's terms); inner solves to rtol and cut to 2 V-cycles;
    # the monodomain reaction explicit (IMEX, Sec. 5.4)
    pf = {}
    for name, mk, u0f in (("heat", si.paper_heat1d, si.u0_paper_heat1d),
                          ("monodomain", si.paper_monodomain, si.u0_paper_monodomain)):
        for M in (1, 2, 3, 4, 5):
            prob = mk(M)
            u0 = torch.as_tensor(u0f(prob)).to(dev)
            for inner in (0, 2):
                h = stmg.Handle(prob, device=dev, pfasst_levels=3, pfasst_inner_cycles=inner, rtol=1e-9,
                                max_cycles=300)
                U = torch.zeros(h.shape, dtype=torch.float64, device=dev)
                _, st, t = _timed_pfasst(h, u0, U)
                pf["%s_M%d_Nt%d%s" % (name, M, prob["N"], "_inner2" if inner else "")] = {
                    "ms": 1e3 * t, "status": st["status"], "iterations": st["cycles"], "rel_res": st["rel_res"]}
                del h, U
    return {"heat_Nx1024_to_1e-9": heat, "heat_weak_Nt_SMGL_V33_fgmres10_to_1e-9": weak,
            "monodomain_SMG7_V33_fgmres10_to_1e-9": mono, "pfasst3_1_to_1e-9": pf}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path (--gpus %d)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import stmg_inputs as si
    from paper_2006_12883_amd import stmg

    dev = torch.device("cuda:0")
    prob = si.config("rd2d")
    u0n = si.initial("rd2d", prob)
    u0 = torch.as_tensor(u0n).to(dev)
    shape = (prob["N"], prob["M"], 256, 256)
    dof = float(np.prod(shape))
    if a.krylov_only:
        print(json.dumps({"krylov_rd2d_fp64_to_1e-10": krylov_lines(dev)}), flush=True)
        return
    if a.only:
        print(json.dumps(extras(dev, a.only)), flush=True)
        return
    if a.kernel_only or a.cycle_only:
        h = stmg.Handle(prob, device=dev)
        U = torch.randn(shape, dtype=torch.float64, device=dev)
        kernels, cyc_ms, lv, c_ms, cbytes, fused0 = time_kernels(h, U, u0, a.kernel_iters)
        cb, _ = cycle_bytes(lv, fused0=fused0)
        print(json.dumps({"kernels": kernels, "vcycle_ms": cyc_ms, "vcycle_bytes": cb,
                          "copy_ms": c_ms, "copy_bytes": cbytes, "copy_GBs": cbytes / c_ms / 1e6}))
        return

    h = stmg.Handle(prob, device=dev)
    U = torch.zeros(shape, dtype=torch.float64, device=dev)
    for _ in range(a.warmup):
        U.zero_()
        h.solve(u0, U)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)
    cycles = 0
    rels = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        U.zero_()
        _, st = h.solve(u0, U)
        cycles += st["cycles"]
        rels.append(st["rel_res"])
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    value = dof * cycles / t
    ms_per_step = 1e3 * t / a.steps
    print("timed solves done", file=sys.stderr, flush=True)

    # time to a 1e-10 residual: FP64 vs mixed precision
    ttr = {}
    sols = {"solve_fp64_rtol1e-12": U.cpu().numpy()}
    for prec in ("fp64", "mixed"):
        hh = stmg.Handle(prob, device=dev, precision=prec, rtol=1e-10)
        V = torch.zeros(shape, dtype=torch.float64, device=dev)
        hh.solve(u0, V)
        best = None
        for _ in range(3):
            V.zero_()
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            _, st = hh.solve(u0, V)
            torch.cuda.synchronize()
            el = time.perf_counter() - s0
            if best is None or el < best[0]:
                best = (el, st)
        ttr[prec] = {"seconds": best[0], "cycles": best[1]["cycles"], "rel_res": best[1]["rel_res"],
                     "refinements": best[1]["refinements"]}
        sols["solve_" + prec + "_rtol1e-10"] = V.cpu().numpy()
        hh.close()
        del V
    # the Krylov option on the same workload, kept for the error check
    hk = stmg.Handle(prob, device=dev, krylov=5, rtol=1e-10)
    V = torch.zeros(shape, dtype=torch.float64, device=dev)
    hk.solve(u0, V)
    sols["solve_fp64_fgmres5_rtol1e-10"] = V.cpu().numpy()
    hk.close()
    del V
    print("time-to-1e-10 done", file=sys.stderr, flush=True)

    # the V-cycle's kernels and whole cycles against the HBM roofline
    kernels, cyc_ms, lv, c_ms, cbytes, fused0 = time_kernels(h, U, u0, a.kernel_iters)
    cb, per_level = cycle_bytes(lv, fused0=fused0)
    cb2, _ = cycle_bytes(lv)
    mb = model_cycle_bytes(lv)
    dom = max((k for k in kernels if kernels[k]["in_cycle"]), key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    achieved = kd["GBs"]
    print("kernel timing done", file=sys.stderr, flush=True)

    out = {
        "metric": "space-time DOF*V-cycles/s (FP64 STMG solve to 1e-12) + time-to-1e-10 residual, mixed vs FP64, 1 GPU",
        "value": value,
        "unit": "DOF*V-cycles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random Fourier modes, |k| <= 16, variance 1/|k|^2)",
        "config": {"workload": "2D linear reaction-diffusion nu=1e-2 lambda=1, periodic 256x256, "
                               "M=3, N=256, T=1, FP64 solve to 1e-12",
                   "dof": int(dof), "cycles_per_solve": cycles / a.steps,
                   "final_rel_res": max(rels)},
        "time_to_1e-10": ttr,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom),
                     "kernel": dom + " (level 0, the longest kernel of the V-cycle)",
                     "kernel_ms": kd["ms"], "bytes_per_launch": kd["bytes"],
                     "level0_kernels": kernels,
                     "cycle_ms": cyc_ms, "cycle_bytes": cb, "cycle_bytes_per_level": per_level,
                     "cycle_GBs": cb / (cyc_ms * 1e-3) / 1e9,
                     "cycle_frac": cb / (cyc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     # priced at the bytes of separate level-0 sweep and restriction kernels
                     "cycle_bytes_separate_level0": cb2,
                     "cycle_frac_separate_level0": cb2 / (cyc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "copy_GBs_smoother_bytes": cbytes / (c_ms * 1e-3) / 1e9,
                     # the same cycle priced at the unfused per-unit word counts:
                     # the fusions save the difference to cycle_bytes
                     "cycle_bytes_unfused_model": mb,
                     "cycle_frac_unfused_model": mb / (cyc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not a.no_extras:
        del h, U
        torch.cuda.empty_cache()
        out["other_workloads"] = extras(dev)
    if not a.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, u0n, sols, ms_per_step * 1e-3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
