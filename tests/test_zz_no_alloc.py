"""The allocation-free FP32 Stokes apply (fsi_apply_stokes_f32_noalloc), called
through the C ABI, against the existing entry point fsi_apply_stokes_f32 on the
same inputs: two calls in a row, the second on a smaller level, so that a stale
staging array from the first call would show; in the phased launch form (bitwise
equal) and in the single atomic launch (equal up to the order of the FP32 adds).
Levels beyond the staging limit are rejected before any work."""
import ctypes as C

import numpy as np
import pytest

from paper_2305_08986_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _vp(t):
    return C.c_void_p(t.data_ptr())


def _pair(ctx, level, seed):
    """(noalloc v, q), (fsi_apply_stokes_f32 v, q) on random FP32 inputs of the level."""
    s = ctx.sizes(level)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    u = torch.rand(s["n_vel"], dtype=torch.float32, device="cuda", generator=g) * 2 - 1
    p = torch.rand(s["n_p"], dtype=torch.float32, device="cuda", generator=g) * 2 - 1
    # outputs pre-filled with garbage: every entry must be written
    v1 = torch.full_like(u, 7.0)
    q1 = torch.full_like(p, -3.0)
    v2 = torch.full_like(u, 5.0)
    q2 = torch.full_like(p, 9.0)
    st = ctx.lib.fsi_apply_stokes_f32_noalloc(ctx.h, level, _vp(u), _vp(p), _vp(v1), _vp(q1))
    assert st == 0, ctx.lib.fsi_last_error(ctx.h)
    st = ctx.lib.fsi_apply_stokes_f32(ctx.h, level, _vp(u), _vp(p), _vp(v2), _vp(q2))
    assert st == 0, ctx.lib.fsi_last_error(ctx.h)
    torch.cuda.synchronize()
    return (v1, q1), (v2, q2)


def _close(a, b, tol):
    a = a.double()
    b = b.double()
    err = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    ent = float((a - b).abs().max() / b.abs().max())
    assert err <= tol and ent <= tol, (err, ent)


@pytest.mark.parametrize("name", ["T3_8", "T2_R"])
def test_noalloc_stokes_f32_matches_the_allocating_entry_point(name):
    from paper_2305_08986_amd import fsi
    wl = W.make_workload(name)
    ctx = fsi.Context.from_mesh(wl.mesh)
    fsi.setup_workload(ctx, wl)
    J = ctx.n_levels - 1
    # phased launches (untuned context): the same kernels on the same inputs, bit for bit
    for level, seed in ((J, 1), (J - 1, 2)):
        (v1, q1), (v2, q2) = _pair(ctx, level, seed)
        assert torch.equal(v1, v2) and torch.equal(q1, q2), (name, level)
    if wl.mesh.dim == 3:
        # the single atomic launch on both levels: equal up to the order of the FP32 adds
        for level in (J, J - 1):
            ctx.set_tuning(level, 1, fsi.ATOMIC_VARIANTS[1])
        ctx.set_mg_params(tuned=1, atomics=1)
        for level, seed in ((J, 3), (J - 1, 4)):
            (v1, q1), (v2, q2) = _pair(ctx, level, seed)
            _close(v1, v2, 1e-6)
            _close(q1, q2, 1e-6)
    ctx.close()


def test_noalloc_rejects_levels_beyond_the_staging_limit():
    """A 2048 x 2048 level has 2049^2 > 2^22 pressure nodes: FSI_ERR_ARG, and no work."""
    from paper_2305_08986_amd import fsi
    ctx = fsi.Context(2, (2048, 2048), (1.0, 1.0), (2048, 2048), W.default_dirichlet_faces(2))
    assert ctx.sizes(0)["n_p"] > (1 << 22)
    dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
    st = ctx.lib.fsi_apply_stokes_f32_noalloc(ctx.h, 0, _vp(dummy), _vp(dummy), _vp(dummy), _vp(dummy))
    assert st == fsi.FSI_ERR_ARG
    assert b"staging limit" in ctx.lib.fsi_last_error(ctx.h)
    torch.cuda.synchronize()
    assert torch.equal(dummy, torch.zeros_like(dummy))
    ctx.close()
