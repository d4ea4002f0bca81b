"""Host-side checks of bench.py: the single-GPU contract and the work model."""

import subprocess
import sys

import bench
import numpy as np


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       cwd=bench.ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stage_work_is_sum_of_kernel_parts():
    for N in range(0, 9):
        Fs, _ = bench.stage_work(N)
        Ft, _ = bench.kernel_work("trace", N)
        Fst, _ = bench.kernel_work("stage", N)
        assert Fs == Ft + Fst


def test_traffic_record_requires_matching_sources():
    assert bench.recorded_traffic("stage", "no such workload") is None
    v = bench.recorded_traffic("stage", "k1d=40 N=4 fp64 fused")
    assert v is None or v > 0


def test_advection_work_is_one_field_of_the_acoustic_contractions():
    for N in range(0, 9):
        Np, n1 = bench.n_basis(N), N + 1
        Nc, Nfc = n1 ** 3, 5 * n1 ** 2
        # trace: the same V^f contraction on one field instead of four
        assert 4 * bench.adv_work("trace", N)[0] == bench.kernel_work("trace", N)[0]
        # stage contractions: three derivatives, projection and lift of one field
        F, B = bench.adv_work("stage", N)
        assert F - (10 * Nc + 8 * Nfc + 6 * Np) == 2 * (3 * Nc * Np + Nc * Np + Nfc * Np)
        assert B == 32 * Np + 8 * n1 ** 2 + 152


def test_plane_wave_dot_matches_matmul():
    import numpy as np
    P = np.random.default_rng(0).standard_normal((7, 5, 3))
    k = np.array([1.5, -0.2, 0.7])
    assert np.allclose(bench._dot3(P, k), P @ k, rtol=1e-15, atol=1e-15)


def test_cpu_baseline_closure_holds_every_face_neighbour():
    """The CPU baseline evaluates the oracle on a sub-mesh made of its sample
    and their neighbours: every face neighbour of a sampled element must be in
    it, so the sampled right-hand sides equal those on the whole mesh."""
    import bench
    from oracle import AcousticDG
    from synth import hex_pyramid_mesh, random_state
    xyz, e2v = hex_pyramid_mesh(4, seed=3)
    K = e2v.shape[0]
    S = np.sort(np.random.default_rng(1).choice(K, 40, replace=False))
    xs, es, loc, sub = bench._face_closure(xyz, e2v, S)
    assert np.array_equal(sub[loc], S)
    U = random_state(K, 2, seed=4)
    full = AcousticDG(xyz, e2v, 2, elems=S).rhs(U)
    part = AcousticDG(xs, es, 2, elems=loc).rhs(U[sub])
    assert np.abs(full - part).max() <= 1e-14 * np.abs(full).max()


def test_headline_takes_the_faster_fp64_path():
    dense = {"value": 17.0, "roofline": {"frac": 0.5}}
    sf = {"value": 31.0, "roofline": {"frac": 0.2}}
    res, path = bench.fp64_headline(dense, {"fp64_sum_factorized": sf})
    assert res is sf and path == "sumfact"
    res, path = bench.fp64_headline({"value": 40.0}, {"fp64_sum_factorized": sf})
    assert res["value"] == 40.0 and path == "fused"


def test_sum_factorised_work_is_below_the_dense_work():
    # the collapsed tensor structure costs O(N^4) per element against O(N^6)
    for N in range(2, 9):
        Fsf, Bsf = bench.sf_work("stage", N, local=True)
        Fd, Bd = bench.kernel_work("stage", N)
        assert Fsf < Fd and Bsf <= Bd
    assert bench.work("stage", 5, "sumfact") == bench.sf_work("stage", 5, local=True)
    assert bench.work("stage", 6, "sumfact") == bench.sf_work("stage", 6, local=False)
