#!/usr/bin/env python3
"""Throughput of the DG acoustics hot path on one MI355X.

One bench step is one LSRK(5,4) time step: five stages, each a full
right-hand side (trace, volume, surface + lift, inverse mass) and the RK
update, over every element of the mesh.  Default workload (the precision-form
configuration): the unit cube as 64^3 perturbed hexahedra x 6 = 1 572 864
pyramids (seed 3), N = 5 (Np = 91), four fields, c = 1, wall boundaries,
penalty flux; initial data the L2-projected wall eigenmode of number m, with
m chosen per N so that the FP64 error lies above the single-precision floors
(equal-error comparison, Section 4.3); then the same for N = 6 and 7.

Prints one JSON line.  ``value`` is GDOF.stages/s = 4 Np K * 5 * steps / t of
the faster of the two FP64 kernel paths at the headline N (dense matrix-core
operators, or the sum-factorised kernels of Section 4.4; both under
``fp64_paths``, each with its roofline: the matrix-core stage against the
FP64 matrix peak, the sum-factorised one against the FP64 vector peak).  The
line carries for the FP32-MFMA and split-BF16 forms their throughput,
roofline (FP32 against its matrix-core peak, split-BF16 against HBM), L2
error against the exact mode, whether the form is at equal error (within
10 % of the FP64 error), its speed-up over the dense FP64 path and over the
faster FP64 path, and the CPU oracle's throughput on all host cores (at most
16) and on one.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GDOF·stages/s, FP64 plain vs FP32-MFMA form at equal L2 error, N=3–7"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0


def n_basis(N):
    return (N + 1) * (N + 2) * (2 * N + 3) // 6


def kernel_work(name: str, N: int):
    """Algorithmic flops and HBM bytes per element for one launch of a kernel.

    Flops count what the method computes (dense operators of Algorithms 1-3);
    bytes count the FP64 data the method must move through HBM (state in and
    out, quad-base traces, 15 vertex doubles, neighbour ids and material).
    """
    Np, n1 = n_basis(N), N + 1
    Nc, Nfc, Nab = n1 ** 3, 5 * n1 ** 2, n1 ** 2
    if name == "trace":            # U^f = V^f U on every face, 4 fields
        return 8 * Nfc * Np, 32 * Np + 32 * Nab
    if name == "volume":           # [Dr;Ds;Dt] U, pointwise metric, V^T (W .)
        return 32 * Nc * Np + 40 * Nc, 32 * Np + 32 * Np + 120
    if name == "surface_update":   # flux, LIFT, inverse mass, LSRK
        return 8 * Nfc * Np + 25 * Nfc + 24 * Np, 32 * Np * 5 + 32 * Nab + 152
    if name == "stage":            # volume + surface + inverse mass + LSRK, fused
        return (32 * Nc * Np + 40 * Nc + 8 * Nfc * Np + 25 * Nfc + 24 * Np,
                32 * Np * 4 + 32 * Nab + 152)
    raise KeyError(name)


def sf_work(name: str, N: int, local: bool = True):
    """Flops and HBM bytes per element of one launch of a sum-factorised
    kernel: the multiply-adds of its one-dimensional contractions (a-, b- and
    c-directions), pointwise metric and fluxes, and the FP64 data it must move
    with traces kept as (p, u.n) pairs -- base faces only when whole
    hexahedra share a workgroup (local); otherwise the four-field traces of
    all five faces from the matrix-core trace kernel."""
    n1 = N + 1
    n2, Np, KJ = n1 * n1, n_basis(N), n1 * (n1 + 1) // 2
    if name == "trace":
        if not local:  # the matrix-core trace kernel, four fields at every face point
            return kernel_work("trace", N)
        return 2 * 4 * n1 * (Np + KJ + n1 * KJ), 32 * Np + 16 * n2
    if name == "stage":
        per_field = (2 * n1 * Np + 4 * n1 * (Np + KJ + n2) + n2 * (3 * KJ + 3 * n2 + 3 * n1)
                     + KJ * n2 + 5 * n1 * Np)
        fma = (4 * per_field + n2 * (9 * n1 + 3 * n2) + 3 * n2 * n1 + n2 * (n2 + 4 * n1)
               + 8 * n1 * n2)
        return 2 * fma, 128 * Np + (16 if local else 160) * n2 + 152
    raise KeyError(name)


def work(name: str, N: int, path: str = "fused"):
    """Per-element work of one launch of kernel ``name`` on kernel path ``path``."""
    # the sum-factorised stage owns whole hexahedra up to N = 5 (the bench
    # meshes come in hexahedra), else it reads all-face traces
    return sf_work(name, N, local=N <= 5) if path == "sumfact" else kernel_work(name, N)


def stage_work(N: int):
    """Whole-stage algorithmic flops and bytes per element."""
    Np, n1 = n_basis(N), N + 1
    Nc, Nfc, Nab = n1 ** 3, 5 * n1 ** 2, n1 ** 2
    F = 32 * Nc * Np + 16 * Nfc * Np + 40 * Nc + 25 * Nfc + 24 * Np
    B = 128 * Np + 64 * Nab + 152
    return F, B


def kernel_sources_digest():
    """SHA-256 over every device source of the library (the .hip and .hpp files
    of csrc/, not the host builders): a traffic record is used only while the
    kernels it was measured on are unchanged."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1502_07703_amd", "csrc")
    for path in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    (copy-calibrated) for this kernel and workload, or None when no record
    exists or the kernel sources changed since the counters were taken."""
    import glob
    digest = kernel_sources_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                rec = json.loads(line.split(":", 1)[1])
                if (rec.get("kernel") == kernel and rec.get("workload") == workload
                        and rec.get("sources_sha256") == digest):
                    return int(rec["bytes_per_launch"])
    return None


def wall_mode_values(P, m, t, out=None, chunk=65536):
    """Exact wall eigenmode of the unit cube, (p, u, v, w) at points P (K, Nc, 3)
    as a (K, 4, Nc) tensor: p = C cos(w t), u_k = sin(w t)/sqrt(3) times the
    mode's k-th gradient factor, C = cos(m pi x) cos(m pi y) cos(m pi z),
    w = sqrt(3) m pi.  Evaluated in element chunks to bound temporaries."""
    import torch
    k = m * np.pi
    om = np.sqrt(3.0) * k
    a = np.sin(om * t) / np.sqrt(3.0)
    K = P.shape[0]
    if out is None:
        out = torch.empty((K, 4, P.shape[1]), dtype=P.dtype, device=P.device)
    for e0 in range(0, K, chunk):
        x, y, z = (P[e0:e0 + chunk, :, d] for d in range(3))
        cx, cy, cz = torch.cos(k * x), torch.cos(k * y), torch.cos(k * z)
        o = out[e0:e0 + chunk]
        o[:, 0] = cx * cy * cz * np.cos(om * t)
        o[:, 1] = a * torch.sin(k * x) * cy * cz
        o[:, 2] = a * cx * torch.sin(k * y) * cz
        o[:, 3] = a * cx * cy * torch.sin(k * z)
    return out


def l2_norm(solver, U, P, wJ, mode=None, chunk=65536):
    """sqrt(sum_q w_q J_q |U(x_q) - f_q|^2) over all fields on the volume rule;
    f is the wall mode (m, t) = ``mode`` or zero."""
    import torch
    vals = solver.evaluate(U)
    tot = 0.0
    for e0 in range(0, vals.shape[0], chunk):
        d = vals[e0:e0 + chunk]
        if mode is not None:
            d = d - wall_mode_values(P[e0:e0 + chunk], mode[0], mode[1])
        tot += float((wJ[e0:e0 + chunk, None, :] * d * d).sum().item())
    del vals
    return float(np.sqrt(tot))


def _host_model():
    """CPU model name of this host (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _host_cores():
    """Cores this process may use, capped at 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _face_closure(xyz, e2v, S):
    """Sub-mesh of the sample S and every element sharing three or more
    vertices with the sample's vertex set (a superset of the face
    neighbours): returns (xyz_sub, e2v_sub, local ids of S, global ids)."""
    Vs = np.unique(e2v[S])
    cnt = np.isin(e2v, Vs).sum(axis=1)
    sub = np.union1d(S, np.nonzero(cnt >= 3)[0])
    uniq, inv = np.unique(e2v[sub], return_inverse=True)
    return xyz[uniq], inv.reshape(-1, 5).astype(np.int64), np.searchsorted(sub, S), sub


def _oracle_worker(args):
    """One worker of the CPU baseline: the oracle's right-hand side on its
    sample of elements (BLAS limited to one thread), timed after a barrier so
    that all workers run at once.  Returns (dof, median seconds)."""
    xyz, e2v, N, loc, U, reps, barrier, queue = args
    from threadpoolctl import threadpool_limits

    from oracle import AcousticDG
    with threadpool_limits(1):
        o = AcousticDG(xyz, e2v, N, elems=loc)
        o.rhs(U)  # warm-up
        if barrier is not None:
            barrier.wait()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            o.rhs(U)
            times.append(time.perf_counter() - t0)
    queue.put((4 * n_basis(N) * loc.size, float(np.median(times))))


def cpu_baseline(xyz, e2v, N, per_worker, workers, reps=3, seed=2024):
    """The oracle (test infrastructure, as it stands) timed on this host's
    cores: ``workers`` processes, each evaluating one right-hand side on its
    own seeded sample of ``per_worker`` elements (plus their face neighbours
    as context), ``reps`` times after a common barrier.  Throughput is the workers' total
    DOF over the slowest worker's median time (they run concurrently).  Runs
    in fresh processes (spawn) before this process touches the GPU."""
    import multiprocessing as mp
    from synth import random_state
    K = e2v.shape[0]
    rng = np.random.default_rng(seed)
    S_all = rng.choice(K, min(per_worker * workers, K), replace=False)
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(workers) if workers > 1 else None
    queue = ctx.Queue()
    procs = []
    for w in range(workers):
        S = np.sort(S_all[w::workers])
        xs, es, loc, sub = _face_closure(xyz, e2v, S)
        U = random_state(es.shape[0], N, seed=seed + w)
        p = ctx.Process(target=_oracle_worker, args=((xs, es, N, loc, U, reps, barrier, queue),))
        p.start()
        procs.append(p)
    res = [queue.get() for _ in procs]
    for p in procs:
        p.join()
    dof = sum(r[0] for r in res)
    t = max(r[1] for r in res)
    return {"value": dof / t / 1e9, "unit": "GDOF·stages/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} x {per_worker} of {K} elements (seeded), one right-hand side "
                      f"(= one stage) each, concurrently, median of {reps}; BLAS 1 thread per "
                      f"process; host: {_host_model()}, {os.cpu_count()} CPUs visible"}


def timed_steps(dg, solver, U, R, t0, dt, nsteps, stream):
    """nsteps LSRK steps through dgpyr_step_timed: wall seconds (bracketed by
    device synchronisation) and per-kernel-kind HIP-event times."""
    import ctypes

    import torch
    L = dg._binding.lib()
    names = L.dgpyr_kernel_names(solver._h).decode().split(";")
    nk = len(names)
    ms = (ctypes.c_double * nk)()
    cnt = (ctypes.c_int64 * nk)()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    st = L.dgpyr_step_timed(solver._h, ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(R.data_ptr()),
                            t0, dt, nsteps, ctypes.c_void_p(stream.cuda_stream), nk, ms, cnt)
    dg._binding.check(st, "dgpyr_step_timed")
    torch.cuda.synchronize()
    return time.perf_counter() - w0, names, list(ms), list(cnt)


def precision_study(args):
    """FP64 vs FP32-MFMA vs split-BF16 on one mesh for several N and modes m:
    throughput of each form and its L2 error against the exact mode and
    against the FP64 result after the same steps (equal error: within 10 % of
    the FP64 error).  Prints one JSON line per (N, m) and a summary line."""
    import torch

    import paper_1502_07703_amd as dg
    from synth import hex_pyramid_mesh
    xyz, e2v = hex_pyramid_mesh(args.study_k1d, seed=3)
    K = e2v.shape[0]
    stream = torch.cuda.current_stream()
    rows = []
    for N in [int(x) for x in args.study_N.split(",")]:
        Np = n_basis(N)
        for m in [int(x) for x in args.study_modes.split(",")]:
            res = {"N": N, "m": m, "nelems": K, "steps": args.study_steps}
            ref_state = None
            for form in ("fp64", "fp32_mfma", "split_bf16"):
                print(f"[study] N={N} m={m} {form}", file=sys.stderr, flush=True)
                with dg.Solver(xyz, e2v, N, precision=form) as s:
                    P, wJ = s.volume_points()
                    U = s.project(wall_mode_values(P, m, 0.0))
                    R = s.empty_state().zero_()
                    dt = s.stable_dt(0.5)
                    wall, names, ms, cnt = timed_steps(dg, s, U, R, 0.0, dt, args.study_steps,
                                                       stream)
                    T_end = args.study_steps * dt
                    e = l2_norm(s, U, P, wJ, (m, T_end))
                    entry = {"gdof_stages_per_s": 4 * Np * K * 5 * args.study_steps / wall / 1e9,
                             "l2_error_vs_mode": e,
                             "kernels_ms": {nm: ms[i] / max(cnt[i], 1) for i, nm in enumerate(names)}}
                    if form == "fp64":
                        ref_state = U.clone()
                        res["t"] = T_end
                    else:
                        entry["l2_diff_vs_fp64"] = l2_norm(s, U - ref_state, P, wJ)
                    del P, wJ
                res[form] = entry
                torch.cuda.empty_cache()
            e64 = res["fp64"]["l2_error_vs_mode"]
            for form in ("fp32_mfma", "split_bf16"):
                f = res[form]
                f["speedup_vs_fp64"] = f["gdof_stages_per_s"] / res["fp64"]["gdof_stages_per_s"]
                f["equal_error"] = abs(f["l2_error_vs_mode"] - e64) <= 0.1 * e64
            print(json.dumps({"study": "precision_forms", **res}), flush=True)
            rows.append(res)
            del ref_state
            torch.cuda.empty_cache()
    return rows


def batch_bench(args):
    """Batched form: independent problems of uneven size (K1D ~ U{lo..hi}
    hexes per side, x 6 pyramids) and order (N ~ U{2..6}), per-element c^2 ~
    U[0.5, 2], one Ricker point source (f0 = 10) at a random location each;
    all advanced together (per-problem CFL time steps) through one captured
    step graph, then the same problems one at a time for comparison.  Prints
    one JSON line."""
    import torch

    import paper_1502_07703_amd as dg
    from synth import hex_pyramid_mesh
    rng = np.random.default_rng(4000)
    lo, hi = [int(x) for x in args.batch_k1d.split(",")]
    probs = []
    for i in range(args.batch_problems):
        k1d = int(rng.integers(lo, hi + 1))
        N = int(rng.integers(2, 7))
        xyz, e2v = hex_pyramid_mesh(k1d, seed=4000 + i)
        K = e2v.shape[0]
        kap = rng.uniform(0.5, 2.0, K)
        src = [dict(x=list(rng.uniform(0.1, 0.9, 3)), f0=10.0)]
        probs.append(dict(xyz=xyz, e2v=e2v, N=N, rho=np.ones(K), kappa=kap, sources=src))
    t_setup = time.perf_counter()
    b = dg.Batch(probs, cfl=0.5)
    t_setup = time.perf_counter() - t_setup
    print(f"[batch] setup {t_setup:.1f} s, {len(probs)} problems, {b.ngroups} groups",
          file=sys.stderr, flush=True)
    U = b.empty_state().zero_()
    R = b.empty_state().zero_()
    stream = torch.cuda.current_stream()
    chosen = b.tune(2)
    b.step(U, R, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(U, R, args.steps, step0=args.warmup)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not torch.isfinite(U).all():
        print("non-finite batch state", file=sys.stderr)
        sys.exit(1)
    dof = sum(4 * sl["Np"] * sl["nelems"] for sl in b.slots)
    nel = sum(sl["nelems"] for sl in b.slots)
    b.close()
    del U, R
    torch.cuda.empty_cache()
    # the same problems one at a time, each in a context of its own with the
    # sum-factorised FP64 kernels and the same steps: the rate the batch
    # replaces
    t_single = 0.0
    for p in probs:
        with dg.Solver(p["xyz"], p["e2v"], p["N"], rho=p["rho"], kappa=p["kappa"],
                       sources=p["sources"], sum_factorized=True) as s1:
            dt1 = s1.stable_dt(0.5)
            U1, R1 = s1.empty_state().zero_(), s1.empty_state().zero_()
            s1.step(U1, R1, dt1, args.warmup)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s1.step(U1, R1, dt1, args.steps, t0=args.warmup * dt1)
            torch.cuda.synchronize()
            t_single += time.perf_counter() - t1
            del U1, R1
    single = dof * 5 * args.steps / t_single / 1e9
    print(f"[batch] batched {dof * 5 * args.steps / wall / 1e9:.2f}, one problem at a time "
          f"{single:.2f} GDOF-stages/s", file=sys.stderr, flush=True)
    out = {"metric": "GDOF·stages/s, batched independent problems", "value":
           dof * 5 * args.steps / wall / 1e9, "unit": "GDOF·stages/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{len(probs)} independent problems, K1D ~ U{{{lo}..{hi}}} x 6 "
                                  "pyramids, N ~ U{2..6}, c^2 ~ U[0.5,2] per element, one Ricker "
                                  "source each, per-problem CFL 0.5 time steps",
                      "problems": len(probs), "nelems": nel, "dof": dof, "groups": b.ngroups,
                      "tuned_shapes": chosen, "setup_s": t_setup},
           "one_problem_at_a_time": {"value": single, "unit": "GDOF·stages/s",
                                     "kernels": "sum-factorised FP64, one context per problem",
                                     "batch_speedup": dof * 5 * args.steps / wall / 1e9 / single}}
    print(json.dumps(out), flush=True)


def _dot3(P, k):
    """P (..., 3) . k (3 numbers), elementwise (no BLAS call on huge shapes)."""
    return float(k[0]) * P[..., 0] + float(k[1]) * P[..., 1] + float(k[2]) * P[..., 2]


def adv_work(name: str, N: int):
    """Algorithmic flops and HBM bytes per element for one launch of an
    advection kernel (one field): trace V^f u; stage [Dr;Ds;Dt] u, pointwise
    beta . adj metric, V^T (W .), face term, LIFT, inverse mass, LSRK."""
    Np, n1 = n_basis(N), N + 1
    Nc, Nfc, Nab = n1 ** 3, 5 * n1 ** 2, n1 ** 2
    if name == "trace":
        return 2 * Nfc * Np, 8 * Np + 8 * Nab
    if name == "stage":
        return (8 * Nc * Np + 2 * Nfc * Np + 10 * Nc + 8 * Nfc + 6 * Np,
                32 * Np + 8 * Nab + 152)
    raise KeyError(name)


def advection_bench(args):
    """Second workload (Section 4.1): u_t + div(beta u) = 0, beta = (1, 0.3,
    -0.5), upwind flux, on the periodic bi-unit cube cut into K1D^3 x 6
    perturbed pyramids; initial data sin(pi (x + y)) projected on the device;
    CFL 0.5 time steps.  One JSON line per N with throughput, kernel times,
    the stage kernel's roofline and the L2 error against the transported
    wave."""
    import torch

    import paper_1502_07703_amd as dg
    from synth import hex_pyramid_mesh, periodic_pair_ids
    beta = np.array([1.0, 0.3, -0.5])
    kv = np.pi * np.array([1.0, 1.0, 0.0])
    xyz, e2v = hex_pyramid_mesh(args.advection_k1d, seed=2, lo=-1.0, hi=1.0)
    pid = periodic_pair_ids(xyz)
    K = e2v.shape[0]
    stream = torch.cuda.current_stream()
    for N in [int(x) for x in args.advection_N.split(",")]:
        Np = n_basis(N)
        print(f"[advection] N={N} K={K}", file=sys.stderr, flush=True)
        with dg.Advection(xyz, e2v, N, beta, alpha=1.0, pair_ids=pid) as s:
            P, wJ = s.volume_points()
            U = s.project(torch.sin(_dot3(P, kv)).unsqueeze(1).contiguous())
            R = s.empty_state().zero_()
            dt = s.stable_dt(0.5)
            s.step(U, R, dt, args.warmup)
            wall, names, ms, cnt = timed_steps(dg, s, U, R, args.warmup * dt, dt,
                                               args.advection_steps, stream)
            T = (args.warmup + args.advection_steps) * dt
            f = s.evaluate(U)[:, 0]
            exact = torch.sin(_dot3(P - torch.from_numpy(beta * T).cuda(), kv))
            err = float(torch.sqrt((wJ * (f - exact) ** 2).sum()))
            del P, wJ, f, exact
        kernels = {}
        for i, nm in enumerate(names):
            avg = ms[i] / max(cnt[i], 1)
            F, Bb = adv_work(nm, N)
            kernels[nm] = {"avg_ms": avg, "launches": int(cnt[i]),
                           "tflops": F * K / (avg * 1e-3) / 1e12,
                           "gbs": Bb * K / (avg * 1e-3) / 1e9}
        F, Bb = adv_work("stage", N)
        t = kernels["stage"]["avg_ms"] * 1e-3
        mf = F / (PEAK_FP64_TFLOPS * 1e12) >= Bb / (PEAK_HBM_GBS * 1e9)
        if mf:
            roof = {"bound": "mfma", "achieved": F * K / t / 1e12, "peak": PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": Bb * K / t / 1e9, "peak": PEAK_HBM_GBS,
                    "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = None
        stages = 5 * args.advection_steps
        out = {"metric": "GDOF·stages/s, advection", "value": Np * K * stages / wall / 1e9,
               "unit": "GDOF·stages/s", "n_gpus": 1, "steps": args.advection_steps,
               "warmup": args.warmup, "ms_per_step": wall / args.advection_steps * 1e3,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": f"periodic bi-unit cube, {args.advection_k1d}^3 perturbed "
                                      f"hexes x 6 = {K} pyramids, N={N}, 1 field, upwind flux, "
                                      "beta = (1, 0.3, -0.5), LSRK(5,4)",
                          "nelems": K, "N": N, "Np": Np, "dof": K * Np, "dt": dt,
                          "l2_error_vs_transported_wave": err},
               "kernels": kernels, "roofline": roof}
        print(json.dumps(out), flush=True)
        torch.cuda.empty_cache()


def adjoint_bench(args):
    """Adjoint form: gradient of a receiver misfit with respect to per-element
    c^2 (kappa, rho = 1) through the discrete adjoint.  K1D^3 x 6 pyramids,
    c^2 = 1 + 0.3 F(x) with F a seeded sum of Fourier modes (|k|_inf <= 4,
    max |F| = 1) at element centroids, one Ricker source at a seeded point
    whose frequency fits the simulated window (f0 = 4 / T, delay 1 / f0,
    T = steps x dt) and seeded receivers on the sphere of radius 0.3 T around
    it (the wave passes them inside the window), data recorded with c^2 = 1,
    checkpoints every few steps.  Prints one JSON line with the forward and
    gradient times."""
    import torch

    import paper_1502_07703_amd as dg
    from paper_1502_07703_amd.adjoint import receiver_misfit
    from synth import hex_pyramid_mesh
    xyz, e2v = hex_pyramid_mesh(args.adjoint_k1d, seed=5)
    K = e2v.shape[0]
    N = args.N if args.N is not None else 4  # the adjoint configuration's order
    rng = np.random.default_rng(5000)
    cent = xyz[e2v].mean(axis=1)
    F = np.zeros(K)
    for _ in range(12):
        k = rng.integers(-4, 5, 3)
        F += rng.normal() * np.cos(2 * np.pi * (cent @ k) + rng.uniform(0, 2 * np.pi))
    c2 = 1.0 + 0.3 * F / np.abs(F).max()
    nsteps, every = args.adjoint_steps, args.adjoint_checkpoint
    # the CFL step of the model c^2 (the larger sound speed: stable for c = 1 too)
    with dg.Solver(xyz, e2v, N, alpha=args.adjoint_alpha, kappa=c2) as s0:
        dt = s0.stable_dt(0.5)
    T = nsteps * dt
    xs = rng.uniform(0.4, 0.6, 3)
    src = [dict(x=list(xs), f0=4.0 / T)]
    d = rng.normal(size=(args.adjoint_receivers, 3))
    rec = xs + 0.3 * T * d / np.linalg.norm(d, axis=1, keepdims=True)
    # forward stages on the sum-factorised kernels (the faster FP64 path); the
    # transposed operator runs on the matrix-core adjoint kernels
    s = dg.Solver(xyz, e2v, N, alpha=args.adjoint_alpha, sources=src, adjoint=True,
                  sum_factorized=True)
    s.set_receivers(rec)
    U0 = s.empty_state().zero_()
    # data: the receiver traces of the true model c^2 = 1
    with torch.no_grad():
        s.set_kappa(np.ones(K))
        U = U0.clone()
        R = s.empty_state().zero_()
        data = torch.empty((nsteps, s.nrec), dtype=torch.float64, device="cuda")
        for n in range(nsteps):
            s.step(U, R, dt, 1, t0=n * dt)
            s.sample_receivers(U, data[n])
    kap = torch.tensor(c2, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = receiver_misfit(kap, s, U0, data, dt, nsteps, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = kap.grad.numpy()
    Np = n_basis(N)
    dof = 4 * Np * K
    # central differences of the misfit on seeded directions (forward runs only)
    fd = []
    rng_d = np.random.default_rng(5100)
    for i in range(args.adjoint_fd_directions):
        d = rng_d.normal(size=K)
        h = 1e-4
        with torch.no_grad():
            Jp = float(receiver_misfit(torch.tensor(c2 + h * d), s, U0, data, dt, nsteps,
                                       every).item())
            Jm = float(receiver_misfit(torch.tensor(c2 - h * d), s, U0, data, dt, nsteps,
                                       every).item())
        fdv, adv = (Jp - Jm) / (2 * h), float(g @ d)
        fd.append({"fd": fdv, "adjoint": adv, "rel_diff": abs(fdv - adv) / abs(fdv)})
        print(f"[adjoint] direction {i}: fd {fdv:.12e} adjoint {adv:.12e}", file=sys.stderr,
              flush=True)
    out = {"metric": "gradient of a receiver misfit w.r.t. per-element c^2 (discrete adjoint)",
           "value": dof * 5 * nsteps / (t2 - t0) / 1e9, "unit": "GDOF·stages/s of forward run",
           "n_gpus": 1, "steps": nsteps, "warmup": 0, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{args.adjoint_k1d}^3 x 6 = {K} pyramids, N={N}, c^2 = 1 + "
                                  f"0.3 F(x), flux alpha = {args.adjoint_alpha:g}, walls, "
                                  f"Ricker source f0 = {4.0 / T:.4g}, receivers on a sphere "
                                  f"of radius {0.3 * T:.3g} around it, "
                                  f"{s.nrec} receivers, {nsteps} steps, checkpoints every "
                                  f"{every}", "nelems": K, "N": N, "dof": dof, "dt": dt,
                      "kernels": "forward sum-factorised, transposed operator on matrix cores"},
           "forward_s": t1 - t0, "gradient_s": t2 - t1, "misfit": float(J.item()),
           "gradient_norm": float(np.linalg.norm(g)), "gradient_finite": bool(np.isfinite(g).all()),
           "central_differences": {"h": 1e-4, "directions": fd,
                                   "max_rel_diff": max((x["rel_diff"] for x in fd), default=None)}}
    s.close()
    print(json.dumps(out), flush=True)


FORM_PEAK = {"fp64": PEAK_FP64_TFLOPS, "fp32_mfma": PEAK_FP32_TFLOPS}
FORM_DTYPE = {"fp64": "f64", "fp32_mfma": "f32 contractions, f64 state",
              "split_bf16": "bf16x3 contractions, f64 state"}
# Wall-eigenmode number per N at which every form reaches equal L2 error on the
# 64^3 x 6 mesh (the FP64 error lies well above the FP32 and split-BF16 floors;
# measured with --study: N = 5, m = 32: 9.1e-6; N = 6, m = 48: 1.1e-5;
# N = 7, m = 64: 7.0e-6, all three forms within 10 %).
EQUAL_ERROR_MODE = {3: 16, 4: 32, 5: 32, 6: 48, 7: 64}


def roofline(kernel, N, K, avg_ms, form, path, traffic):
    """Roofline object of one kernel: algorithmic flops (or bytes) per launch
    over its average HIP-event duration, against the peak that binds it.
    FP64 and FP32 contraction kernels: their matrix-core peak (compute-bound at
    these orders); split-BF16: HBM, since its three bf16 products per
    multiply-add take less time at the bf16 peak than its bytes at 8 TB/s;
    the sum-factorised FP64 stage: whichever of its vector-ALU flops at the
    FP64 peak and its bytes at 8 TB/s takes longer."""
    F, Bb = work(kernel, N, path)
    t = avg_ms * 1e-3
    per = {"flop": F * K, "bytes": Bb * K}
    compute_bound = F / (PEAK_FP64_TFLOPS * 1e12) >= Bb / (PEAK_HBM_GBS * 1e9)
    if form == "split_bf16" or not compute_bound:
        ach = Bb * K / t / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "kernel": kernel,
                "per_launch": per}
    ach = F * K / t / 1e12
    peak = FORM_PEAK[form]
    return {"bound": "mfma" if path in ("fused", "unfused") else "alu", "achieved": ach,
            "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic,
            "kernel": kernel, "per_launch": per}


def run_form(dg, xyz, e2v, k1d, N, form, mode, steps, warmup, stream, path="fused", groups=0,
             trace_groups=0, lds_operators=None, keep_state=False):
    """One precision form / kernel path on one mesh: projected wall mode m,
    ``warmup`` untimed steps, ``steps`` timed steps (dgpyr_step_timed), L2 error
    against the exact mode at the final time.  Returns a result dict (and the
    final state and the cubature points when keep_state)."""
    import torch
    K = e2v.shape[0]
    Np = n_basis(N)
    print(f"[bench] N={N} {form} {path} K={K} m={mode}", file=sys.stderr, flush=True)
    t_setup = time.perf_counter()
    s = dg.Solver(xyz, e2v, N, precision=form, reference_kernels=path == "reference",
                  unfused=path == "unfused", sum_factorized=path == "sumfact",
                  groups_per_wave=groups, trace_groups=trace_groups, lds_operators=lds_operators)
    t_setup = time.perf_counter() - t_setup
    P, wJ = s.volume_points()
    U = s.project(wall_mode_values(P, mode, 0.0))
    R = s.empty_state().zero_()
    dt = s.stable_dt(0.5)
    s.step(U, R, dt, warmup)
    torch.cuda.synchronize()
    wall, names, ms, cnt = timed_steps(dg, s, U, R, warmup * dt, dt, steps, stream)
    if not torch.isfinite(U).all():
        print(f"non-finite state after the timed steps ({form}, N={N})", file=sys.stderr)
        sys.exit(1)
    stages = 5 * steps
    kernels = {}
    for i, nm in enumerate(names):
        avg = ms[i] / max(cnt[i], 1)
        F, Bb = work(nm, N, path)
        kernels[nm] = {"avg_ms": avg, "launches": int(cnt[i]),
                       "tflops": F * K / (avg * 1e-3) / 1e12,
                       "gbs": Bb * K / (avg * 1e-3) / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    g = s.info_groups()
    traffic = recorded_traffic(dom, f"k1d={k1d} N={N} {form} {path} g{g}")
    T_end = (warmup + steps) * dt
    Fs_, Bs_ = work(dom, N, path)
    res = {"value": 4 * Np * K * stages / wall / 1e9, "ms_per_step": wall / steps * 1e3,
           "hbm_frac_dominant": Bs_ * K / (kernels[dom]["avg_ms"] * 1e-3) / (PEAK_HBM_GBS * 1e9),
           "dt": dt, "t_end": T_end, "setup_s": t_setup, "groups_per_wave": g,
           "l2_error_vs_mode": l2_norm(s, U, P, wJ, (mode, T_end)),
           "roofline": roofline(dom, N, K, kernels[dom]["avg_ms"], form, path, traffic),
           "kernels": kernels}
    Fs, Bs = stage_work(N)
    t_stage = wall / stages
    res["stage"] = {"flop_per_stage": Fs * K, "bytes_per_stage": Bs * K,
                    "tflops": Fs * K / t_stage / 1e12, "gbs": Bs * K / t_stage / 1e9,
                    "frac_fp64_roof": (Fs * K / t_stage) / (PEAK_FP64_TFLOPS * 1e12),
                    "frac_hbm_roof": (Bs * K / t_stage) / (PEAK_HBM_GBS * 1e9)}
    if keep_state:
        return res, s, U, P, wJ
    s.close()
    del U, R, P, wJ
    torch.cuda.empty_cache()
    return res


def fp64_headline(dense, forms):
    """The faster FP64 path of one order (dense matrix-core operators or sum
    factorisation) and its kernel-path name."""
    sf = forms["fp64_sum_factorized"]
    return (sf, "sumfact") if sf["value"] > dense["value"] else (dense, "fused")


def _path_summary(res):
    keys = ("value", "ms_per_step", "roofline", "kernels", "l2_error_vs_mode")
    return {k: res[k] for k in keys if k in res}


def compare_forms(dg, xyz, e2v, k1d, N, mode, steps, warmup, stream):
    """FP64 and both precision forms on one mesh and mode, and the FP64
    sum-factorised kernels: each one's result with its speed-up over the
    dense FP64 path (the same operators in FP64) and over the faster FP64
    path, its L2 distance to the FP64 state and whether it is at equal error
    (within 10 % of the FP64 error)."""
    import torch
    base, s64, U64, P, wJ = run_form(dg, xyz, e2v, k1d, N, "fp64", mode, steps, warmup, stream,
                                     keep_state=True)
    forms = {}
    for form, path in (("fp32_mfma", "fused"), ("split_bf16", "fused"), ("fp64", "sumfact")):
        res, sf, Uf, _, _ = run_form(dg, xyz, e2v, k1d, N, form, mode, steps, warmup, stream,
                                     path=path, keep_state=True)
        res["speedup_vs_fp64"] = res["value"] / base["value"]
        res["l2_diff_vs_fp64"] = l2_norm(sf, Uf - U64, P, wJ)
        e64 = base["l2_error_vs_mode"]
        res["equal_error"] = abs(res["l2_error_vs_mode"] - e64) <= 0.1 * e64
        sf.close()
        del Uf
        torch.cuda.empty_cache()
        forms[form if path == "fused" else "fp64_sum_factorized"] = res
    best = max(base["value"], forms["fp64_sum_factorized"]["value"])
    for res in forms.values():
        res["speedup_vs_fp64_best"] = res["value"] / best
    s64.close()
    del U64, P, wJ
    torch.cuda.empty_cache()
    return base, forms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--k1d", type=int, default=64)
    ap.add_argument("--N", type=int, default=None,
                    help="order (default 5 for the headline line, 4 for --adjoint)")
    ap.add_argument("--extra-N", default="6,7",
                    help="further orders run after the headline one (comma list, '' for none)")
    ap.add_argument("--mode", type=int, default=0,
                    help="wall eigenmode number m of the initial data (0: the equal-error mode "
                         "of each N)")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--single", action="store_true",
                    help="time one path (--precision and the kernel flags) only")
    ap.add_argument("--reference-kernels", action="store_true",
                    help="plain FP64 vector-ALU kernels instead of the matrix-core ones")
    ap.add_argument("--unfused", action="store_true",
                    help="separate matrix-core volume and surface launches")
    ap.add_argument("--sum-factorized", action="store_true",
                    help="FP64 sum-factorised kernels")
    ap.add_argument("--groups", type=int, default=0,
                    help="4-element groups per wave of the fused matrix-core kernels "
                         "(0 = library default)")
    ap.add_argument("--trace-groups", type=int, default=0,
                    help="4-element groups per wave of the trace kernel (0 = library default)")
    ap.add_argument("--lds-operators", type=int, default=-1,
                    help="1: stage operator tiles in LDS per workgroup, 0: do not, "
                         "-1: library default")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy a 256 MiB buffer 3 times (a plain copy "
                         "of known size for scaling HBM counters)")
    ap.add_argument("--cpu-per-worker", type=int, default=4096,
                    help="elements per CPU worker in the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", action="store_true",
                    help="batched independent problems instead of the bench line")
    ap.add_argument("--batch-problems", type=int, default=256)
    ap.add_argument("--batch-k1d", default="4,24")
    ap.add_argument("--adjoint", action="store_true",
                    help="adjoint-form gradient run instead of the bench line")
    ap.add_argument("--adjoint-k1d", type=int, default=32)
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--adjoint-checkpoint", type=int, default=20)
    ap.add_argument("--adjoint-receivers", type=int, default=64)
    ap.add_argument("--adjoint-alpha", type=float, default=1.0,
                    help="flux parameter of the adjoint run (1: the flux of Section 4.3)")
    ap.add_argument("--adjoint-fd-directions", type=int, default=10,
                    help="central-difference checks of the adjoint gradient (0: none)")
    ap.add_argument("--advection", action="store_true",
                    help="advection workload (Section 4.1) instead of the bench line")
    ap.add_argument("--advection-k1d", type=int, default=64)
    ap.add_argument("--advection-N", default="1,2,3,4,5,6")
    ap.add_argument("--advection-steps", type=int, default=20)
    ap.add_argument("--study", action="store_true",
                    help="precision-form study instead of the bench line (see --study-*)")
    ap.add_argument("--study-k1d", type=int, default=64)
    ap.add_argument("--study-N", default="5,6,7")
    ap.add_argument("--study-modes", default="1,8")
    ap.add_argument("--study-steps", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is "
              "single-device and is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    from synth import hex_pyramid_mesh
    headline = not (args.study or args.batch or args.adjoint or args.advection)
    N = args.N if args.N is not None else 5
    xyz = e2v = None
    cpu = cpu1 = None
    if headline:
        xyz, e2v = hex_pyramid_mesh(args.k1d, seed=3 if args.k1d == 64 else 2)
        if not args.no_cpu_baseline:
            # the oracle on the host cores, before this process touches the GPU
            cores = _host_cores()
            print(f"[bench] CPU baseline: oracle on {cores} cores, then 1", file=sys.stderr,
                  flush=True)
            cpu = cpu_baseline(xyz, e2v, N, args.cpu_per_worker, cores)
            cpu1 = cpu_baseline(xyz, e2v, N, args.cpu_per_worker, 1)

    import torch

    import paper_1502_07703_amd as dg

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.study:
        precision_study(args)
        return
    if args.batch:
        batch_bench(args)
        return
    if args.adjoint:
        adjoint_bench(args)
        return
    if args.advection:
        advection_bench(args)
        return
    K = e2v.shape[0]
    Np = n_basis(N)
    stream = torch.cuda.current_stream()
    mode = args.mode or EQUAL_ERROR_MODE.get(N, 1)
    path = ("reference" if args.reference_kernels else "sumfact" if args.sum_factorized
            else "unfused" if args.unfused else "fused")
    workload = (f"unit cube, {args.k1d}^3 perturbed hexes x 6 = {K} pyramids, N={N}, 4 fields, "
                f"walls, penalty flux, LSRK(5,4), projected wall eigenmode m={mode}")
    if args.single or path != "fused" or args.precision != "fp64":
        main_res = run_form(dg, xyz, e2v, args.k1d, N, args.precision, mode, args.steps,
                            args.warmup, stream, path=path, groups=args.groups,
                            trace_groups=args.trace_groups,
                            lds_operators=None if args.lds_operators < 0 else bool(args.lds_operators))
        forms, orders = None, {}
    else:
        dense, forms = compare_forms(dg, xyz, e2v, args.k1d, N, mode, args.steps, args.warmup,
                                     stream)
        # the headline FP64 figure is the faster of the two FP64 kernel paths
        # (dense matrix-core operators, sum factorisation); both are reported
        main_res, path = fp64_headline(dense, forms)
        orders = {}
        for n2 in [int(x) for x in args.extra_N.split(",") if x.strip()]:
            m2 = EQUAL_ERROR_MODE.get(n2, 1)
            b2, f2 = compare_forms(dg, xyz, e2v, args.k1d, n2, m2, args.steps, args.warmup,
                                   stream)
            orders[str(n2)] = {"mode": m2, "fp64": b2, **f2,
                               "fp64_faster_path": fp64_headline(b2, f2)[1]}
            print(f"[bench] N={n2}: fp64 {b2['value']:.2f}, " + ", ".join(
                f"{k} {v['value']:.2f}" for k, v in f2.items()) + " GDOF-stages/s",
                file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "GDOF·stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": FORM_DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": workload, "k1d": args.k1d, "nelems": K, "N": N, "Np": Np,
                   "dof": 4 * Np * K, "precision": args.precision, "stages_per_step": 5,
                   "dt": main_res["dt"], "mode": mode,
                   "groups_per_wave": main_res["groups_per_wave"],
                   "kernels": {"reference": "reference (vector ALU)",
                               "sumfact": "sum-factorised, fused", "unfused":
                               "matrix core, unfused", "fused": "matrix core, fused"}[path]},
        "roofline": main_res["roofline"],
        "stage": main_res["stage"],
        "kernels": main_res["kernels"],
        "l2_error_vs_mode": {"mode": mode, "t": main_res["t_end"],
                             "value": main_res["l2_error_vs_mode"]},
    }
    if forms is not None:
        out["fp64_paths"] = {"matrix_core_fused": _path_summary(dense),
                             "sum_factorized": _path_summary(forms["fp64_sum_factorized"])}
        out["precision_forms"] = forms
        out["orders"] = orders
    if args.copy_calibration:
        nbytes = 256 << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes, "launches": 3}
    if cpu is not None:
        out["cpu_baseline"] = cpu
        out["cpu_baseline_1core"] = cpu1
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
