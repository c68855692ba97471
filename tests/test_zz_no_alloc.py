"""isb_hessvec_noalloc, the Hessian-vector product for callers that cannot allocate, against
isb_hessvec (the same product with library-allocated staging) and against the FP64 oracle's
assembled Hessian: two calls in a row on one GPU, the second on a smaller mesh, in both precisions
and both scatter paths (LDS-staged patches on the large body, per-corner atomics on the small one),
plus the size limit of the fixed scratch."""
import numpy as np
import pytest

from tests.gpu_util import problems, rand_workload, rel

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _case(dim, shape, seed, precision):
    from paper_2102_05791_amd import Context
    w, rng = rand_workload(dim, seed=seed, shape=shape)
    ctx = Context.from_workload(w, precision=precision, scatter=2)
    x = w.x0 + 0.05 * rng.normal(size=w.x0.shape)
    pv = rng.normal(size=x.shape)
    return w, ctx, x, pv, w.actions[1]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_noalloc_hessvec_matches_hessvec_twice_second_smaller(precision, tol):
    import torch
    cases = [_case(3, (16, 16, 11), 61, precision),   # 16,896 tets: patch scatter
             _case(2, (40, 13), 62, precision)]       # 1,040 triangles (ragged tail): atomic scatter
    for w, ctx, x, pv, a in cases:
        print(f"noalloc {precision} dim {w.dim} n_e {w.T.shape[0]}", flush=True)
        ref = ctx.hessvec(_dev(x), _dev(w.x0), _dev(a), _dev(pv))
        out = torch.full_like(ref, float("nan"))
        ctx.hessvec_noalloc(_dev(x), _dev(w.x0), _dev(a), _dev(pv), out)
        torch.cuda.synchronize()
        ref, out = ref.cpu().numpy(), out.cpu().numpy()
        assert np.all(np.isfinite(out))
        # same kernels: only the order of the FP64 atomic additions may differ
        assert rel(out, ref) <= 1e-12
        assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
        p = problems(w)[0]
        H = p.hessian(x, w.x0, a)
        hp = H @ pv.ravel()
        assert rel(out.ravel(), hp, abs(H) @ np.abs(pv.ravel())) <= tol


def test_noalloc_hessvec_rejects_a_mesh_beyond_its_scratch():
    from paper_2102_05791_amd import Context, IsbError, isb
    from synth import meshes, scenes
    X, T = meshes.tri_grid(1300, 700)      # 912,001 vertices: 36.5 MB of staging > 32 MiB
    ctx = Context(0, "fp64")
    ctx.mesh_upload(2, X, T)
    n_e = T.shape[0]
    mu, lam = scenes.lame(1e4, 0.3)
    f = np.zeros((n_e, 2))
    f[:, 0] = 1.0
    ctx.material_upload(np.full(n_e, mu), np.full(n_e, lam), np.full(n_e, 1e4), f, np.ones(n_e),
                        scenes.scene("be", h=1.0 / 60.0))
    x = _dev(X)
    with pytest.raises(IsbError) as e:
        ctx.hessvec_noalloc(x, x, _dev(np.ones(n_e)), x, _dev(np.zeros_like(X)))
    assert e.value.status == isb.ISB_E_ARG
    assert "scratch" in str(e.value)
