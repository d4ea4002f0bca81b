"""Build and run the CPU emulation of the sum-factorised kernels.

The library's kernel source is compiled for the host with g++, AddressSanitizer
and UndefinedBehaviorSanitizer against the stand-in hip/hip_runtime.h of this
folder (every work item an OS thread, workgroup barriers real barriers), so that its
indexing and its results can be checked without a GPU.  Test infrastructure
only.

    python tests/cpu_emu/run.py --k1d 40 --N 4    # one right-hand side on a mesh
    python tests/cpu_emu/run.py --k1d 64 --N 5 --edge-blocks 64
        # the first and last 64 workgroups of each launch only (index check)
"""

from __future__ import annotations

import argparse
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1502_07703_amd", "csrc")
EXE = os.path.join(ROOT, "_build", "emu_sumfact")
SOURCES = [os.path.join(HERE, "emu_sumfact.cpp"), os.path.join(CSRC, "host", "refops.cpp"),
           os.path.join(CSRC, "host", "mesh.cpp")]
DEPS = SOURCES + [os.path.join(CSRC, n) for n in
                  ("kernels_sumfact.hip", "context.hpp", "flux.hpp", "geom.hpp")] + \
    [os.path.join(HERE, "hip", "hip_runtime.h"), os.path.abspath(__file__)]


def build(force: bool = False) -> str:
    """Compile the emulator (g++, address and undefined-behaviour sanitizers) if it is missing or stale."""
    if not force and os.path.exists(EXE):
        t = os.path.getmtime(EXE)
        if all(os.path.getmtime(d) <= t for d in DEPS):
            return EXE
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    tmp = f"{EXE}.{os.getpid()}.tmp"
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-pthread", f"-I{HERE}", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *SOURCES,
           "-o", tmp]
    # Parallel test workers may build at once: each writes its own file and
    # renames it into place, so no worker ever runs a half-written binary.
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("emulator build failed:\n" + r.stderr[-4000:])
    os.replace(tmp, EXE)
    return EXE


def run(xyz, e2v, N, U, rho=None, kappa=None, bc="wall", alpha=1.0, nsteps=0, dt=0.0,
        timeout=3600, edge_blocks=0):
    """Right-hand side (nsteps = 0) or the state after nsteps LSRK steps,
    shape (K, 4, Np), and whether the whole-hexahedron variant ran."""
    exe = build()
    K = e2v.shape[0]
    Np = (N + 1) * (N + 2) * (2 * N + 3) // 6
    rho = np.ones(K) if rho is None else np.asarray(rho, dtype=np.float64)
    kappa = np.ones(K) if kappa is None else np.asarray(kappa, dtype=np.float64)
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fin, "wb") as f:
            np.array([N, xyz.shape[0], K, {"wall": 0, "free": 1}[bc], nsteps],
                     dtype=np.int64).tofile(f)
            np.array([alpha, dt], dtype=np.float64).tofile(f)
            np.ascontiguousarray(xyz, dtype=np.float64).tofile(f)
            np.ascontiguousarray(e2v, dtype=np.int64).tofile(f)
            rho.astype(np.float64).tofile(f)
            kappa.astype(np.float64).tofile(f)
            np.ascontiguousarray(U, dtype=np.float64).tofile(f)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
        if edge_blocks:
            env["EMU_EDGE_BLOCKS"] = str(edge_blocks)
        r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=timeout,
                           env=env)
        if r.returncode != 0:
            raise RuntimeError(f"emulator exit {r.returncode}:\n{r.stderr[-6000:]}")
        raw = np.fromfile(fout, dtype=np.float64, offset=8)
        local = bool(np.fromfile(fout, dtype=np.int64, count=1)[0])
    return raw.reshape(K, 4, Np), local


def main():
    sys.path.insert(0, ROOT)
    from synth import hex_pyramid_mesh, random_state
    ap = argparse.ArgumentParser()
    ap.add_argument("--k1d", type=int, default=40)
    ap.add_argument("--N", type=int, default=4)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--edge-blocks", type=int, default=0)
    a = ap.parse_args()
    xyz, e2v = hex_pyramid_mesh(a.k1d, seed=a.seed)
    U = random_state(e2v.shape[0], a.N, seed=11)
    t = time.time()
    out, local = run(xyz, e2v, a.N, U, edge_blocks=a.edge_blocks)
    part = f"first and last {a.edge_blocks} workgroups" if a.edge_blocks else "every workgroup"
    print(f"k1d={a.k1d} N={a.N} K={e2v.shape[0]} ({part}): finite={bool(np.isfinite(out).all())} "
          f"whole-hexahedron={local} {time.time() - t:.1f} s, no sanitizer report")


if __name__ == "__main__":
    main()
