"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: FP64 right-hand side within 1e-12 relative to the oracle, per field
(max abs difference over all coefficients / max abs oracle value), in the
canonical coefficient layout; LSRK trajectories within 1e-11.
"""

import numpy as np
import pytest

from gpu_helpers import gpu_rhs, log, rel_err_per_field
from oracle import AcousticDG, lsrk_run
from oracle.dg import wall_mode
from synth import hex_pyramid_mesh, octahedron_mesh, random_materials, random_state, single_pyramid

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _solver(xyz, e2v, N, **kw):
    import paper_1502_07703_amd as dg
    return dg.Solver(xyz, e2v, N, **kw)


PATHS = {"mfma": {}, "sumfact": {"sum_factorized": True}}
# matrix-core dense operators, and the sum-factorised kernels (whole
# hexahedra per workgroup where the mesh allows, N <= 6; otherwise traces of
# all faces through HBM)
PATH_PARAMS = [pytest.param("mfma"), pytest.param("sumfact")]
# 4-element groups per wave exercised per path (the fused matrix-core kernels
# take 1 or 2; 0 = the library's default).
GROUPS = {"mfma": (1, 2), "sumfact": (0,)}


@pytest.mark.parametrize("path", PATH_PARAMS)
@pytest.mark.parametrize("N", list(range(0, 9)))
def test_rhs_parity_cfg1_all_orders(N, path):
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=N)
    U = random_state(K, N, seed=100 + N)
    log(f"[parity] cfg1 N={N} K={K} path={path}")
    ref = AcousticDG(xyz, e2v, N, rho=rho, kappa=kap).rhs(U)
    for g in GROUPS[path]:
        with _solver(xyz, e2v, N, rho=rho, kappa=kap, groups_per_wave=g, **PATHS[path]) as s:
            got = gpu_rhs(s, U)
        err = rel_err_per_field(got, ref)
        log(f"[parity] cfg1 N={N} groups={g} rel err per field {err}")
        assert np.all(err < TOL), (g, err)


@pytest.mark.parametrize("bc", ["wall", "free"])
@pytest.mark.parametrize("alpha", [0.0, 1.0, 0.37])
def test_rhs_parity_flux_and_bc(bc, alpha):
    N = 3
    xyz, e2v = hex_pyramid_mesh(2, seed=2)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=5)
    U = random_state(K, N, seed=7)
    log(f"[parity] bc={bc} alpha={alpha}")
    ref = AcousticDG(xyz, e2v, N, rho=rho, kappa=kap, bc=bc, alpha=alpha).rhs(U)
    with _solver(xyz, e2v, N, rho=rho, kappa=kap, bc=bc, alpha=alpha) as s:
        got = gpu_rhs(s, U)
    assert np.all(rel_err_per_field(got, ref) < TOL)


@pytest.mark.parametrize("path", PATH_PARAMS)
@pytest.mark.parametrize("N", [2, 4])
def test_rhs_parity_shuffled_mesh(N, path):
    """Element order permuted and base loops rotated: exercises every quad orientation."""
    xyz, e2v = hex_pyramid_mesh(3, seed=3, shuffle=True)
    K = e2v.shape[0]
    U = random_state(K, N, seed=9)
    log(f"[parity] shuffled K={K} N={N} path={path}")
    ref = AcousticDG(xyz, e2v, N).rhs(U)
    with _solver(xyz, e2v, N, **PATHS[path]) as s:
        got = gpu_rhs(s, U)
    assert np.all(rel_err_per_field(got, ref) < TOL)


@pytest.mark.parametrize("path", PATH_PARAMS)
@pytest.mark.parametrize("nsub", [1, 7, 13, 29])
def test_rhs_parity_ragged_subsets(nsub, path):
    """Meshes whose element counts leave partial workgroups (cut faces become walls)."""
    N = 5
    xyz, e2v = hex_pyramid_mesh(2, seed=4)
    e2v = e2v[:nsub]
    U = random_state(nsub, N, seed=nsub)
    log(f"[parity] ragged K={nsub} path={path}")
    ref = AcousticDG(xyz, e2v, N).rhs(U)
    for g in GROUPS[path]:
        with _solver(xyz, e2v, N, groups_per_wave=g, **PATHS[path]) as s:
            got = gpu_rhs(s, U)
        assert np.all(rel_err_per_field(got, ref) < TOL), g


def test_rhs_parity_special_meshes():
    for (xyz, e2v) in (single_pyramid(), octahedron_mesh()):
        for N in (0, 1, 3):
            U = random_state(e2v.shape[0], N, seed=1)
            ref = AcousticDG(xyz, e2v, N).rhs(U)
            with _solver(xyz, e2v, N) as s:
                got = gpu_rhs(s, U)
            assert np.all(rel_err_per_field(got, ref) < TOL)


def test_rhs_parity_eigenmode_data():
    N = 3
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    o = AcousticDG(xyz, e2v, N)
    U = o.project(wall_mode(1), xyz, e2v, t=0.2)
    ref = o.rhs(U)
    with _solver(xyz, e2v, N) as s:
        got = gpu_rhs(s, U)
    assert np.all(rel_err_per_field(got, ref) < TOL)


@pytest.mark.parametrize("groups", [1, 2])
def test_rhs_bitwise_deterministic(groups):
    import torch
    N = 4
    xyz, e2v = hex_pyramid_mesh(3, seed=6)
    U = random_state(e2v.shape[0], N, seed=2)
    with _solver(xyz, e2v, N, groups_per_wave=groups) as s:
        Ud = s.pack(torch.from_numpy(U).cuda())
        a = s.rhs(Ud).clone()
        b = s.rhs(Ud).clone()
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("path", PATH_PARAMS)
@pytest.mark.parametrize("N", [3, 5, 6, 7, 8])
def test_step_parity_lsrk(path, N):
    """Ten LSRK(5,4) steps on the 48-pyramid mesh: GPU trajectory vs oracle
    trajectory, for every build of the in-place stage kernels (N = 5 to 8 are
    compiled for other register budgets and, at N = 7 and 8, spill)."""
    import torch
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    o = AcousticDG(xyz, e2v, N)
    U0 = o.project(wall_mode(1), xyz, e2v)
    dt = 0.5 / (2.0 * (N + 1) * (N + 3) / 3.0 * o.inverse_length().max())
    nsteps = 10
    ref, _ = lsrk_run(o.rhs, U0, dt, nsteps)
    for g in GROUPS[path]:
        with _solver(xyz, e2v, N, groups_per_wave=g, **PATHS[path]) as s:
            U = s.pack(torch.from_numpy(U0).cuda())
            R = s.empty_state().fill_(float("nan"))  # R is never read before it is written
            s.step(U, R, dt, nsteps)
            got = s.unpack(U).cpu().numpy()
        err = rel_err_per_field(got, ref)
        log(f"[parity] LSRK 10 steps N={N} groups={g} rel err {err}")
        assert np.all(err < 1e-11), (g, err)


@pytest.mark.parametrize("path", PATH_PARAMS)
@pytest.mark.parametrize("k1d,N,nsample", [(40, 4, 3000)])
def test_rhs_parity_full_size_sampled(k1d, N, nsample, path):
    """The benchmark workload (40^3 hexes x 6 = 384000 pyramids, N = 4): the GPU
    computes every element; the oracle checks a seeded sample of elements."""
    xyz, e2v = hex_pyramid_mesh(k1d, seed=2)
    K = e2v.shape[0]
    U = random_state(K, N, seed=11)
    rng = np.random.default_rng(12)
    sample = np.unique(np.concatenate([rng.choice(K, nsample, replace=False), [0, K - 1]]))
    log(f"[parity] full-size K={K} N={N} sample={sample.size} path={path}")
    ref = AcousticDG(xyz, e2v, N, elems=sample).rhs(U)
    for g in GROUPS[path]:
        with _solver(xyz, e2v, N, groups_per_wave=g, **PATHS[path]) as s:
            got = gpu_rhs(s, U)
        err = rel_err_per_field(got[sample], ref)
        log(f"[parity] full-size groups={g} rel err {err}")
        assert np.all(err < TOL), (g, err)


@pytest.mark.parametrize("N", [1, 4, 7])
def test_rhs_parity_reference_kernels(N):
    """The plain FP64 vector-ALU kernels (flag) meet the same bar as the default."""
    xyz, e2v = hex_pyramid_mesh(2, seed=8)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=9)
    U = random_state(K, N, seed=10)
    ref = AcousticDG(xyz, e2v, N, rho=rho, kappa=kap).rhs(U)
    with _solver(xyz, e2v, N, rho=rho, kappa=kap, reference_kernels=True) as s:
        got = gpu_rhs(s, U)
    assert np.all(rel_err_per_field(got, ref) < TOL)


@pytest.mark.parametrize("N", [3, 5, 7])
def test_rhs_fp32_mfma_form(N):
    """FP32 matrix-core contractions (volume, lift) with FP64 geometry, traces,
    flux, mass and state: error against the FP64 oracle at the FP32 level."""
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    U = random_state(K, N, seed=3)
    ref = AcousticDG(xyz, e2v, N).rhs(U)
    for g in (1, 2):
        with _solver(xyz, e2v, N, precision="fp32_mfma", groups_per_wave=g) as s:
            got = gpu_rhs(s, U)
        err = rel_err_per_field(got, ref)
        log(f"[fp32] N={N} groups={g} rel err per field {err}")
        assert np.all(err < FP32_BAR), (g, err)
        assert np.any(err > 1e-10), "FP32 form gave FP64-accurate results: wrong kernels?"


@pytest.mark.parametrize("N", [2, 6])
def test_rhs_parity_unfused_matrix_core(N):
    """Separate matrix-core volume and surface launches (flag) meet the same bar."""
    xyz, e2v = hex_pyramid_mesh(2, seed=12)
    K = e2v.shape[0]
    U = random_state(K, N, seed=13)
    ref = AcousticDG(xyz, e2v, N).rhs(U)
    with _solver(xyz, e2v, N, unfused=True) as s:
        got = gpu_rhs(s, U)
    assert np.all(rel_err_per_field(got, ref) < TOL)


# Right-hand-side bars of the precision forms against the FP64 oracle on
# random data (relative, per field), set from the measured errors with a
# margin of about 3.5: FP32-MFMA at most 8.9e-7 (N = 3, 5, 7), split-BF16 at
# most 1.45e-5 (N = 2, 4, 6, 7, 8).
FP32_BAR = 3e-6
BF16_BAR = 5e-5


@pytest.mark.parametrize("N", [2, 4, 6, 7, 8])
def test_rhs_split_bf16_form(N):
    """Split-BF16 matrix-core contractions (three bf16 products per multiply, FP32
    accumulation) with FP64 geometry, traces, flux, mass and state.  Each split
    operand keeps about 16 mantissa bits, so the right-hand side is accurate to
    roughly 1e-5 relative."""
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    U = random_state(K, N, seed=4)
    ref = AcousticDG(xyz, e2v, N).rhs(U)
    with _solver(xyz, e2v, N, precision="split_bf16") as s:
        got = gpu_rhs(s, U)
    err = rel_err_per_field(got, ref)
    log(f"[bf16] N={N} rel err per field {err}")
    assert np.all(err < BF16_BAR), err
    assert np.any(err > 1e-10), "split-BF16 form gave FP64-accurate results: wrong kernels?"


@pytest.mark.parametrize("prec", ["fp32_mfma", "split_bf16"])
@pytest.mark.parametrize("N", [6, 8])
def test_precision_form_lsrk_steps(prec, N):
    """Three LSRK(5,4) steps of each precision form (the in-place stage kernels
    compiled for two waves per SIMD from N = 6, spilling at N = 8) against the
    oracle's FP64 trajectory: the state moves by dt rhs per stage, so the
    error is the right-hand side's bar scaled by dt |rhs| / |U|, bounded here
    by the bar itself."""
    import torch
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    U0 = random_state(K, N, seed=90 + N)
    o = AcousticDG(xyz, e2v, N)
    dt, n = 1e-3, 3
    ref, _ = lsrk_run(o.rhs, U0, dt, n)
    with _solver(xyz, e2v, N, precision=prec) as s:
        U = s.pack(torch.from_numpy(U0).cuda())
        R = s.empty_state().fill_(float("nan"))
        s.step(U, R, dt, n)
        got = s.unpack(U).cpu().numpy()
    err = rel_err_per_field(got, ref)
    log(f"[{prec}] LSRK 3 steps N={N} rel err {err}")
    assert np.all(err < (FP32_BAR if prec == "fp32_mfma" else BF16_BAR)), err
    assert np.any(err > 1e-14), "reduced-precision steps gave FP64-accurate results"


@pytest.mark.parametrize("N", [0, 1, 2, 3, 4, 5, 6])
def test_rhs_parity_operator_staging(N):
    """Operator tiles staged in LDS per workgroup (FP64 up to N = 5, FP32 up to
    N = 6; above that the default kernel runs) on the cfg1 mesh and a ragged
    subset, and one LSRK step."""
    import torch
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    for sub in (48, 29):
        e = e2v[:sub]
        K = e.shape[0]
        rho, kap = random_materials(K, seed=N)
        U = random_state(K, N, seed=60 + N)
        o = AcousticDG(xyz, e, N, rho=rho, kappa=kap)
        ref = o.rhs(U)
        with _solver(xyz, e, N, rho=rho, kappa=kap, lds_operators=True) as s:
            got = gpu_rhs(s, U)
        assert np.all(rel_err_per_field(got, ref) < TOL), (sub, rel_err_per_field(got, ref))
        with _solver(xyz, e, N, rho=rho, kappa=kap, precision="fp32_mfma", lds_operators=True) as s:
            got = gpu_rhs(s, U)
        assert np.all(rel_err_per_field(got, ref) < 2e-5), sub
    dt = 1e-3
    ref, _ = lsrk_run(o.rhs, U, dt, 2)
    with _solver(xyz, e, N, rho=rho, kappa=kap, lds_operators=True) as s:
        Ud = s.pack(torch.from_numpy(U).cuda())
        R = s.empty_state().zero_()
        s.step(Ud, R, dt, 2)
        got = s.unpack(Ud).cpu().numpy()
    assert np.all(rel_err_per_field(got, ref) < 1e-11)


@pytest.mark.parametrize("N", [0, 2, 4, 5, 6])
def test_rhs_parity_trace_groups(N):
    """The trace kernel with 1, 2 and 4 element groups per wave (cfg1 mesh and
    a ragged subset): identical results."""
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    for sub in (48, 13):
        e = e2v[:sub]
        K = e.shape[0]
        U = random_state(K, N, seed=80 + N)
        ref = AcousticDG(xyz, e, N).rhs(U)
        outs = []
        for tg in (1, 2, 4):
            with _solver(xyz, e, N, trace_groups=tg) as s:
                got = gpu_rhs(s, U)
            assert np.all(rel_err_per_field(got, ref) < TOL), (sub, tg)
            outs.append(got)
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
