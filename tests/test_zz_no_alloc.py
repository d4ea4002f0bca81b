"""dgpyr_adjoint_rhs_noalloc (static device scratch, no allocation) against
dgpyr_adjoint_rhs on the same inputs, through the C ABI: two calls in a row,
the second on a smaller context (the shared array keeps the first call's
contents), and the size limit."""

import ctypes

import numpy as np
import pytest

from gpu_helpers import log, rel_err_per_field
from synth import hex_pyramid_mesh, random_materials, random_state

pytestmark = pytest.mark.gpu


def _noalloc(s, lam, out):
    import torch

    from paper_1502_07703_amd import _binding as B
    return B.lib().dgpyr_adjoint_rhs_noalloc(
        s._h, ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_matches_adjoint_rhs():
    import torch

    import paper_1502_07703_amd as dg
    from paper_1502_07703_amd import _binding as B
    # larger context first, then a smaller one with another order
    for k1d, N, alpha, bc in ((3, 4, 1.0, "wall"), (2, 3, 0.37, "free")):
        xyz, e2v = hex_pyramid_mesh(k1d, seed=k1d)
        K = e2v.shape[0]
        rho, kap = random_materials(K, seed=N)
        with dg.Solver(xyz, e2v, N, rho=rho, kappa=kap, alpha=alpha, bc=bc) as s:
            lam = s.pack(torch.from_numpy(random_state(K, N, seed=70 + N)).cuda())
            ref = s.adjoint_rhs(lam)
            got = torch.full_like(ref, float("nan"))
            st = _noalloc(s, lam, got)
            assert st == B.OK, B.lib().dgpyr_last_error()
            torch.cuda.synchronize()
            a = s.unpack(got).cpu().numpy()
            b = s.unpack(ref).cpu().numpy()
        err = rel_err_per_field(a, b)
        log(f"[noalloc] K={K} N={N} rel err per field {err} bitwise {np.array_equal(a, b)}")
        assert np.all(np.isfinite(a))
        assert np.all(err < 1e-12), err


def test_noalloc_rejects_states_beyond_the_scratch():
    """48000 pyramids at N = 4: 4 K Np doubles = 84 MB > 64 MiB -> E_ARG, and
    the output array is left untouched."""
    import torch

    import paper_1502_07703_amd as dg
    from paper_1502_07703_amd import _binding as B
    xyz, e2v = hex_pyramid_mesh(20, seed=1)
    with dg.Solver(xyz, e2v, 4) as s:
        assert s.state_len * 8 > B.NOALLOC_SCRATCH_BYTES
        lam = s.empty_state().zero_()
        out = s.empty_state().fill_(3.0)
        assert _noalloc(s, lam, out) == B.E_ARG
        assert b"exceeds the static scratch" in B.lib().dgpyr_last_error()
        torch.cuda.synchronize()
        assert bool((out == 3.0).all())
