"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Bars (FP64 unless stated):
 * stencil product: every cell within 16 u (sum of |terms|), u = 2^-53;
 * solves: the oracle recomputes ||b - A x|| / ||b|| <= tol for the GPU's x;
   at tol 1e-13 the GPU and oracle solutions agree to 1e-10 relative on
   systems whose condition number keeps that meaningful (cd recipe);
 * pure FP32: the oracle's FP64 residual of the GPU's x <= 1e-5;
 * batched == one-at-a-time, bit for bit;
 * adjoint: lambda and the 7 gradients against dense LAPACK (8^3) and against
   the oracle's own transpose solve and gradient formulas (64^3).
"""
import os

import numpy as np
import pytest

from paper_2211_15605_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2211_15605_amd import binding
    binding.load()  # raises if the HIP library is missing: there is no fallback
    return torch, torch.device("cuda", 0)


def dev_arrays(torch, dev, arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev) for a in arrs]


def host(t):
    return t.detach().cpu().numpy().ravel()


def context(grids, precision="fp64", env=None):
    from paper_2211_15605_amd.solver import Context
    old = {}
    env = env or {}
    for k, v in env.items():
        old[k] = os.environ.get(k)
        os.environ[k] = str(v)
    try:
        return Context(grids, precision=precision)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def abs_terms(orc, shape, diags, x):
    """|a_P x| + sum |a_nb x_nb| per cell (forward operator)."""
    neg = [np.abs(diags[0])] + [-np.abs(d) for d in diags[1:]]
    return orc.apply(shape, neg, np.abs(x))


SHAPES = [(16, 16, 16), (33, 17, 9), (97, 31, 5), (1, 1, 7), (5, 1, 1), (1, 300, 2), (130, 3, 40),
          (64, 64, 4), (200, 7, 3)]
# launch shapes of the multi-kernel path (EQS_SMALL=0 keeps tiny grids off the one-block path)
TILINGS = [dict(EQS_SMALL=0), dict(EQS_SMALL=0, EQS_CPT=1, EQS_KC=1), dict(EQS_SMALL=0, EQS_CPT=2, EQS_KC=3),
           dict(EQS_SMALL=0, EQS_CPT=2, EQS_KC=7)]
# solve paths: the one-block persistent solve (sets of at most 2048 cells, by default), the
# single-sync march iteration (one launch per step) and the three-launch iteration
PATHS = [dict(), dict(EQS_SMALL=0), dict(EQS_SMALL=0, EQS_SYNC=3), dict(EQS_SMALL=0, EQS_UNSCALED=1)]
PATH_IDS = ["small", "sync1", "sync3", "sync1_unscaled"]
# the two march iterations on sets above the one-block size
SCHEMES = [dict(), dict(EQS_SYNC=3)]
SCHEME_IDS = ["sync1", "sync3"]
# launch shapes of the single-sync step: 512-thread blocks over segments of 1024 cells, and tiles
# numbered segment-fastest (each combined with small chunks, so several chunks and tiles per set)
FUSED_SHAPES = [dict(EQS_FNT=512), dict(EQS_FORD=1, EQS_KC=3), dict(EQS_FNT=512, EQS_FORD=1, EQS_KC=5),
                dict(EQS_FNT=512, EQS_CPT=1, EQS_KC=4)]
FUSED_IDS = ["fnt512", "ford1_kc3", "fnt512_ford1_kc5", "fnt512_cpt1_kc4"]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("transpose", [False, True])
def test_apply_matches_oracle_per_cell(torch_dev, orc, shape, transpose):
    torch, dev = torch_dev
    g = W.Grid(*shape)
    diags = W.random_general(g, seed=21)
    x = np.random.default_rng(22).standard_normal(g.n)
    ref = orc.apply(shape, diags, x, transpose)
    bound = 16 * EPS * (abs_terms(orc, shape, diags, x) if not transpose else
                        orc.apply(shape, [np.abs(diags[0])] + [-np.abs(d) for d in diags[1:]], np.abs(x), True))
    for tl in TILINGS:
        ctx = context([shape], env=tl)
        y = host(ctx.apply(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [x])[0], transpose=transpose))
        assert np.all(np.abs(y - ref) <= bound + 1e-300), (tl, np.max(np.abs(y - ref) - bound))
        ctx.close()


def manufactured(orc, cfg, grid=None, recipe=None, set_id=0):
    s = W.make_set(cfg, set_id, grid=grid, recipe=recipe)
    g = s["grid"]
    b = orc.apply(g.shape, s["diags"], s["x_star"])
    return g, s["diags"], b, s["x_star"]


@pytest.mark.parametrize("path", PATHS, ids=PATH_IDS)
def test_fp64_config0_residual_and_iterations(torch_dev, orc, path):
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 0)
    ctx = context([g.shape], env=path)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-10, maxit=1000)
    xg = host(x)
    assert info["status"] == 0
    rel = orc.rel_residual(g.shape, diags, b, xg)
    assert rel <= 1e-10
    assert abs(rel - info["rel_res"]) <= 1e-3 * rel
    _, oinfo = orc.bicgstab(g.shape, diags, b, tol=1e-10, maxit=1000)
    # rounding differs, so iteration counts may differ slightly (parity unpinned)
    assert abs(info["iters"] - oinfo["iters"]) <= 3, (info, oinfo)
    assert np.max(np.abs(xg - xs)) <= orc.forward_error_certificate(g.shape, diags, b, xg) * (1 + 1e-6)


@pytest.mark.parametrize("shape", [(12, 12, 12), (16, 8, 16), (1, 2048, 1), (1, 64, 32), (1, 1, 2049)])
def test_fp64_one_block_path_sizes(torch_dev, orc, shape):
    # the one-block solve up to its 2048-cell limit (and one cell past it, on the march path):
    # the same solution as the oracle, and the same as the march path's
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 0, grid=W.Grid(*shape))
    xo, oinfo = orc.bicgstab(g.shape, diags, b, tol=1e-13, maxit=5000)
    D = dev_arrays(torch, dev, diags)
    bd = dev_arrays(torch, dev, [b])[0]
    out = []
    for env in (dict(), dict(EQS_SMALL=0)):
        ctx = context([g.shape], env=env)
        x, info = ctx.solve(D, bd, tol=1e-13, maxit=5000)
        xg = host(x)
        assert info["status"] == 0, (env, info)
        assert orc.rel_residual(g.shape, diags, b, xg) <= 1e-13
        assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo), env
        out.append(xg)
        ctx.close()
    assert np.linalg.norm(out[0] - out[1]) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("cfg,shape", [(0, (16, 16, 16)), (0, (37, 23, 11)), (3, (64, 64, 64)),
                                       (2, (97, 31, 5)), (0, (130, 3, 40)), (0, (5, 1, 1))])
def test_fp64_matches_oracle_solution(torch_dev, orc, cfg, shape):
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, cfg, grid=W.Grid(*shape))
    xo, oinfo = orc.bicgstab(g.shape, diags, b, tol=1e-13, maxit=5000)
    assert oinfo["status"] == 0
    for tl in [dict(), dict(EQS_SYNC=3)] + TILINGS[:3] + [dict(TILINGS[2], EQS_SYNC=3)] + \
            [dict(f, EQS_SMALL=0) for f in FUSED_SHAPES]:
        ctx = context([g.shape], env=tl)
        x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-13, maxit=5000)
        xg = host(x)
        assert info["status"] == 0, info
        assert orc.rel_residual(g.shape, diags, b, xg) <= 1e-13
        assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo), tl
        ctx.close()


def test_fp64_repeatable_bitwise(torch_dev, orc):
    torch, dev = torch_dev
    g, diags, b, _ = manufactured(orc, 0, grid=W.Grid(40, 30, 20))
    ctx = context([g.shape])
    D = dev_arrays(torch, dev, diags)
    bd = dev_arrays(torch, dev, [b])[0]
    outs = [host(ctx.solve(D, bd, tol=1e-11, maxit=2000)[0]) for _ in range(4)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_graph_replay_equals_eager_launches(torch_dev, orc, precision, scheme):
    # captured iteration chunks are replayed many times, with other device work and
    # synchronisations between calls; every result must equal the eager path's bit for bit
    torch, dev = torch_dev
    g, diags, b, _ = manufactured(orc, 2, grid=W.Grid(33, 65, 20))
    D = dev_arrays(torch, dev, diags)
    bd = dev_arrays(torch, dev, [b])[0]
    eager = context([g.shape], precision=precision, env=dict(scheme, EQS_GRAPHS=0))
    ref, rinfo = eager.solve(D, bd, tol=1e-11, maxit=3000)
    ref = host(ref)
    graphed = context([g.shape], precision=precision, env=scheme)
    for rep in range(4):
        junk = torch.randn(1 << 20, device=dev, dtype=torch.float64).cumsum(0)  # unrelated eager work
        torch.cuda.synchronize()
        x, info = graphed.solve(D, bd, tol=1e-11, maxit=3000)
        assert np.array_equal(host(x), ref), rep
        assert info == rinfo
        del junk


def test_autotune_and_cache_roundtrip(torch_dev, orc, tmp_path):
    torch, dev = torch_dev
    g, diags, b, _ = manufactured(orc, 0, grid=W.Grid(40, 48, 24))
    D = dev_arrays(torch, dev, diags)
    bd = dev_arrays(torch, dev, [b])[0]
    cache = str(tmp_path / "tune.jsonl")
    ctx = context([g.shape])
    lay = ctx.autotune(cache_path=cache, iters=4)[0]
    x, info = ctx.solve(D, bd, tol=1e-10, maxit=2000)
    assert orc.rel_residual(g.shape, diags, b, host(x)) <= 1e-10
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"nx": 40' in lines[0]
    # a new context picks the tuned shape from the cache
    ctx2 = context([g.shape], env=dict(EQS_TUNE_CACHE=cache))
    lay2 = ctx2.layout()
    for k in ("cpt", "kc", "tiles"):
        assert lay2[k] == lay[k], (lay, lay2)
    x2, info2 = ctx2.solve(D, bd, tol=1e-10, maxit=2000)
    assert np.array_equal(host(x2), host(x))


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_autotune_batched_context(torch_dev, orc, precision, tmp_path):
    """Tuning a context of four staggered sets also times their batched launch (one common depth
    for all sets may beat each set's own choice there); whatever it keeps, the batched solve meets
    tol, equals each set's own solve in the same context bit for bit, and the cache holds one
    per-set entry for each grid."""
    torch, dev = torch_dev
    systems = [manufactured(orc, 2, grid=W.Grid(*s), set_id=i) for i, s in enumerate(STAGGERED_SMALL)]
    cache = str(tmp_path / "tune.jsonl")
    ctx = context(STAGGERED_SMALL, precision=precision)
    lays = ctx.autotune(cache_path=cache, iters=4)
    for lay, sh in zip(lays, STAGGERED_SMALL):
        assert lay["tiles"] == lay["segments"] * lay["chunks"] and 1 <= lay["kc"] <= sh[2], lay
        assert lay["chunks"] == -(-sh[2] // lay["kc"]), lay
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=3000)
    for i, sy in enumerate(systems):
        assert infos[i]["status"] == 0, infos[i]
        assert orc.rel_residual(sy[0].shape, sy[1], sy[2], host(xb[i])) <= 1e-10
        xi, info = ctx.solve(Ds[i], bs[i], tol=1e-10, maxit=3000, set_id=i)
        assert np.array_equal(host(xi), host(xb[i])) and info == infos[i], i
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 4 and all('"nx": %d, "ny": %d, "nz": %d' % sh in ln for sh, ln in zip(STAGGERED_SMALL, lines))


@pytest.mark.parametrize("path", PATHS, ids=PATH_IDS)
def test_fp64_status_codes(torch_dev, orc, path):
    torch, dev = torch_dev
    from paper_2211_15605_amd.solver import EqSolveError
    g, diags, b, xs = manufactured(orc, 0, grid=W.Grid(6, 6, 6))
    ctx = context([g.shape], env=path)
    D = dev_arrays(torch, dev, diags)
    bd, xsd = dev_arrays(torch, dev, [b, xs])
    # maxit too small: computed, not converged
    x, info = ctx.solve(D, bd, tol=1e-12, maxit=1, check=False)
    _, oinfo = orc.bicgstab(g.shape, diags, b, tol=1e-12, maxit=1)
    assert info["status"] == 1 and info["iters"] == 1 and oinfo["status"] == 1
    assert abs(info["rel_res"] - oinfo["rel_res"]) <= 1e-8 * oinfo["rel_res"]
    # exact initial guess: no iteration, x untouched
    x0 = xsd.clone()
    x, info = ctx.solve(D, bd, x=x0, tol=1e-10)
    assert info["iters"] == 0 and np.array_equal(host(x), xs)
    # b = 0 gives x = 0
    x, info = ctx.solve(D, torch.zeros_like(bd), x=torch.ones_like(bd), tol=1e-10)
    assert info["status"] == 0 and not np.any(host(x))
    # NaN in b: non-finite, x untouched
    bn = bd.clone(); bn[5] = float("nan")
    x0 = torch.full_like(bd, 3.0)
    x, info = ctx.solve(D, bn, x=x0, check=False)
    assert info["status"] == 3 and np.all(host(x) == 3.0)
    # zero diagonal entry: argument error found on the device, x untouched
    Dz = [d.clone() for d in D]; Dz[0][4] = 0.0
    with pytest.raises(EqSolveError):
        ctx.solve(Dz, bd, x=x0)
    assert np.all(host(x0) == 3.0)
    # bad tolerance rejected before the call
    with pytest.raises(ValueError):
        ctx.solve(D, bd, tol=0.0)


@pytest.mark.parametrize("path", PATHS, ids=PATH_IDS)
def test_fp64_diagonal_system_one_half_step(torch_dev, orc, path):
    torch, dev = torch_dev
    g = W.Grid(9, 8, 7)
    rng = np.random.default_rng(6)
    P = rng.uniform(1, 3, g.n)
    diags = [P] + [np.zeros(g.n)] * 6
    b = rng.uniform(-1, 1, g.n)
    ctx = context([g.shape], env=path)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-12, maxit=10)
    assert info["status"] == 0 and info["iters"] == 1
    np.testing.assert_allclose(host(x), b / P, rtol=4 * EPS, atol=0)


@pytest.mark.parametrize("path", PATHS, ids=PATH_IDS)
def test_fp64_breakdown_integer_system(torch_dev, orc, path):
    torch, dev = torch_dev
    z = np.zeros(2)
    diags = [np.ones(2), np.array([2.0, 0.0]), z, z, z, z, z]
    ctx = context([(2, 1, 1)], env=path)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [np.ones(2)])[0], tol=1e-10,
                        maxit=10, check=False)
    _, oinfo = orc.bicgstab((2, 1, 1), diags, np.ones(2), tol=1e-10, maxit=10)
    assert info["status"] == 2 == oinfo["status"] and info["iters"] == 1 == oinfo["iters"]


@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
@pytest.mark.parametrize("cfg,shape", [(0, (16, 16, 16)), (1, (32, 64, 32)), (2, (49, 97, 23))])
def test_fp32_refine_reaches_fp64_tolerance(torch_dev, orc, cfg, shape, scheme):
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, cfg, grid=W.Grid(*shape))
    ctx = context([g.shape], precision="fp32_refine", env=scheme)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-10, maxit=20000)
    assert info["status"] == 0, info
    assert info["outer"] >= 2
    rel = orc.rel_residual(g.shape, diags, b, host(x))
    assert rel <= 1e-10
    assert abs(rel - info["rel_res"]) <= 1e-3 * rel


@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
def test_fp32_pure_residual(torch_dev, orc, scheme):
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 0)
    ctx = context([g.shape], precision="fp32", env=scheme)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-5, maxit=2000)
    assert info["status"] == 0, info
    assert orc.rel_residual(g.shape, diags, b, host(x)) <= 1e-5
    xo, _ = orc.bicgstab(g.shape, diags, b, tol=1e-13)
    # forward error against the FP64 oracle: bounded by the Varah certificate of
    # the FP32 result (a 1e-5 residual fixes the error only up to the condition number)
    cert = orc.forward_error_certificate(g.shape, diags, b, host(x))
    err = np.max(np.abs(host(x) - xo))
    print("fp32 pure: residual %.2e, max forward error vs oracle %.2e, certificate %.2e" % (
        info["rel_res"], err, cert), flush=True)
    assert err <= cert * (1 + 1e-6) + 1e-12


STAGGERED_SMALL = [(24, 96, 24), (25, 96, 24), (24, 97, 24), (24, 96, 25)]


@pytest.mark.parametrize("scheme", SCHEMES + FUSED_SHAPES, ids=SCHEME_IDS + FUSED_IDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_batched_equals_sequential_bitwise(torch_dev, orc, precision, scheme):
    torch, dev = torch_dev
    systems = [manufactured(orc, 2, grid=W.Grid(*s), set_id=i) for i, s in enumerate(STAGGERED_SMALL)]
    ctx = context(STAGGERED_SMALL, precision=precision, env=scheme)
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=2000)
    for i, s in enumerate(systems):
        xi, info = ctx.solve(Ds[i], bs[i], tol=1e-10, maxit=2000, set_id=i)
        assert np.array_equal(host(xi), host(xb[i])), i
        assert info == infos[i]
        assert orc.rel_residual(s[0].shape, s[1], s[2], host(xb[i])) <= 1e-10


def test_batched_tiny_sets_one_launch(torch_dev, orc):
    # four tiny staggered sets: one block per set, each equal to its own solve
    torch, dev = torch_dev
    shapes = [(8, 16, 8), (9, 16, 8), (8, 17, 8), (8, 16, 9)]
    systems = [manufactured(orc, 2, grid=W.Grid(*sh), set_id=i) for i, sh in enumerate(shapes)]
    ctx = context(shapes)
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    xb, infos = ctx.solve_batched(Ds, bs, tol=1e-12, maxit=2000)
    for i, s in enumerate(systems):
        xi, info = ctx.solve(Ds[i], bs[i], tol=1e-12, maxit=2000, set_id=i)
        assert np.array_equal(host(xi), host(xb[i])) and info == infos[i]
        assert orc.rel_residual(s[0].shape, s[1], s[2], host(xb[i])) <= 1e-12
        xo, _ = orc.bicgstab(s[0].shape, s[1], s[2], tol=1e-13)
        assert np.linalg.norm(host(xb[i]) - xo) <= 1e-9 * np.linalg.norm(xo)


@pytest.mark.parametrize("path", PATHS, ids=PATH_IDS)
def test_adjoint_matches_dense_reference(torch_dev, orc, path):
    torch, dev = torch_dev
    g = W.Grid(8, 8, 8)
    s = W.make_set(3, 0, grid=g, with_weights=True)
    diags, w = s["diags"], s["w"]
    A = orc.dense(g.shape, diags)
    b = A @ s["x_star"]
    x = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, w)
    G = orc.grad(g.shape, lam, x)
    ctx = context([g.shape], env=path)
    D = dev_arrays(torch, dev, diags)
    xd, wd = dev_arrays(torch, dev, [x, w])
    gb, gd, info = ctx.adjoint(D, xd, wd, tol=1e-13, maxit=1000)
    assert info["status"] == 0
    np.testing.assert_allclose(host(gb), lam, rtol=0, atol=1e-10 * np.max(np.abs(lam)))
    for k in range(7):
        np.testing.assert_allclose(host(gd[k]), G[k], rtol=0, atol=1e-10 * np.max(np.abs(G[k])) + 1e-300)


@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
def test_adjoint_config3_matches_oracle(torch_dev, orc, scheme):
    torch, dev = torch_dev
    g = W.Grid(64, 64, 64)
    s = W.make_set(3, 0, grid=g, with_weights=True)
    diags, w = s["diags"], s["w"]
    b = orc.apply(g.shape, diags, s["x_star"])
    xo, _ = orc.bicgstab(g.shape, diags, b, tol=1e-13, maxit=2000)
    lo, linfo = orc.bicgstab(g.shape, diags, w, tol=1e-13, maxit=2000, transpose=True)
    assert linfo["status"] == 0
    Go = orc.grad(g.shape, lo, xo)
    ctx = context([g.shape], env=scheme)
    D = dev_arrays(torch, dev, diags)
    xd, wd = dev_arrays(torch, dev, [xo, w])
    gb, gd, info = ctx.adjoint(D, xd, wd, tol=1e-13, maxit=2000)
    assert info["status"] == 0
    assert orc.rel_residual(g.shape, diags, w, host(gb), transpose=True) <= 1e-13
    assert np.linalg.norm(host(gb) - lo) <= 1e-10 * np.linalg.norm(lo)
    for k in range(7):
        assert np.linalg.norm(host(gd[k]) - Go[k]) <= 1e-10 * np.linalg.norm(Go[k]) + 1e-300, k


def test_autograd_function_backward(torch_dev, orc):
    torch, dev = torch_dev
    from paper_2211_15605_amd.autograd import EqSolveFn
    g = W.Grid(6, 5, 4)
    s = W.make_set(3, 0, grid=g, with_weights=True)
    shp = (g.nz, g.ny, g.nx)
    T = [torch.tensor(d.reshape(shp), device=dev, requires_grad=True) for d in s["diags"]]
    A = orc.dense(g.shape, s["diags"])
    bnp = A @ s["x_star"]
    bt = torch.tensor(bnp.reshape(shp), device=dev, requires_grad=True)
    x = EqSolveFn.apply(*T, bt, None, 1e-13, 1000)
    wt = torch.tensor(s["w"].reshape(shp), device=dev)
    (x * wt).sum().backward()
    xx = np.linalg.solve(A, bnp)
    lam = np.linalg.solve(A.T, s["w"])
    G = orc.grad(g.shape, lam, xx)
    np.testing.assert_allclose(host(bt.grad), lam, rtol=0, atol=1e-10 * np.max(np.abs(lam)))
    for k in range(7):
        np.testing.assert_allclose(host(T[k].grad), G[k], rtol=0, atol=1e-10 * np.max(np.abs(G[k])) + 1e-300)


# ---------------------------------------------------------------- full-size workloads (as benchmarked)

# (the last: a launch layout on which the FP32 single-sync inner iteration once derailed, the
# regression case of the direct-sigma check and of the refinement's weak-step allowance)
@pytest.mark.parametrize("scheme", SCHEMES + [dict(EQS_CPT=2, EQS_KC=16, EQS_FLAT_MAX=256)],
                         ids=SCHEME_IDS + ["sync1_kc16_flat256"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "fp32"])
def test_config1_full_size_residual(torch_dev, orc, precision, scheme):
    # FP64 and FP32 + refinement to 1e-10; pure FP32 (one FP32 solve of the FP64 system) to 1e-5,
    # each in the oracle's FP64 residual of the returned x
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1)
    tol = 1e-5 if precision == "fp32" else 1e-10
    ctx = context([g.shape], precision=precision, env=scheme)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=tol, maxit=20000)
    print("config1", precision, info, ctx.layout(), flush=True)
    assert info["status"] == 0
    xg = host(x)
    rel = orc.rel_residual(g.shape, diags, b, xg)
    assert rel <= tol
    assert np.max(np.abs(xg - xs)) <= orc.forward_error_certificate(g.shape, diags, b, xg) * (1 + 1e-6)


def test_fp32_refine_sigma_restart_budget_is_per_inner_solve(torch_dev, orc):
    # With reruns off, a tight sigma consistency threshold makes the FP32 single-sync iteration
    # restart often.  Each inner solve of the refinement has its own budget of 32 restarts, so a
    # solve whose inner solves restart more than 32 times in all still reaches the FP64 tolerance;
    # the count is reported in info["sigma_restarts"].
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1)
    D = dev_arrays(torch, dev, diags)
    bd = dev_arrays(torch, dev, [b])[0]
    seen = []
    for stol in (3e-4, 1e-4, 3e-5):
        ctx = context([g.shape], precision="fp32_refine", env=dict(EQS_SIGMA_TOL32=stol, EQS_SIGMA_REDO=0))
        x, info = ctx.solve(D, bd, tol=1e-10, maxit=20000, check=False)
        ctx.close()
        print("sigma tol %g:" % stol, info, flush=True)
        seen.append(info["sigma_restarts"])
        if info["sigma_restarts"] > 32:
            assert info["status"] == 0, info
            assert orc.rel_residual(g.shape, diags, b, host(x)) <= 1e-10
            return
    pytest.fail("no threshold forced more than 32 restarts: %s" % seen)


@pytest.mark.parametrize("precision,stol", [("fp32_refine", None), ("fp32_refine", 3e-4), ("fp64", 1e-9)])
def test_sigma_mismatch_reruns_the_step(torch_dev, orc, precision, stol):
    # With EQS_SIGMA_REDO=1 a step whose expanded sigma parts from the directly summed one runs
    # again with alpha from the direct value (no restart): on the near-singular pressure-like
    # system at full size, with the default threshold and with thresholds tight enough to force
    # many reruns, the solve meets 1e-10 in the oracle's residual and restarts never
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1)
    D = dev_arrays(torch, dev, diags)
    bd = dev_arrays(torch, dev, [b])[0]
    env = {} if stol is None else {"EQS_SIGMA_TOL32" if precision != "fp64" else "EQS_SIGMA_TOL": stol}
    ctx = context([g.shape], precision=precision, env=dict(env, EQS_SIGMA_REDO=1))
    x, info = ctx.solve(D, bd, tol=1e-10, maxit=20000, check=False)
    ctx.close()
    print(precision, stol, info, flush=True)
    assert info["status"] == 0 and info["sigma_restarts"] == 0, info
    if stol is not None:
        assert info["sigma_reruns"] > 0, info
    assert orc.rel_residual(g.shape, diags, b, host(x)) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_sigma_reruns_batched_equals_sequential(torch_dev, orc, precision):
    # reruns forced by a tight threshold are per set: the batched call equals the single ones
    torch, dev = torch_dev
    systems = [manufactured(orc, 2, grid=W.Grid(*s), set_id=i) for i, s in enumerate(STAGGERED_SMALL)]
    env = {"EQS_SIGMA_TOL": 1e-14} if precision == "fp64" else {"EQS_SIGMA_TOL32": 1e-5}
    ctx = context(STAGGERED_SMALL, precision=precision, env=dict(env, EQS_SMALL=0, EQS_SIGMA_REDO=1))
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=4000)
    assert sum(i["sigma_reruns"] for i in infos) > 0, infos
    for i, s in enumerate(systems):
        xi, info = ctx.solve(Ds[i], bs[i], tol=1e-10, maxit=4000, set_id=i)
        assert np.array_equal(host(xi), host(xb[i])), i
        assert info == infos[i]
        assert info["sigma_restarts"] == 0
        assert orc.rel_residual(s[0].shape, s[1], s[2], host(xb[i])) <= 1e-10
    ctx.close()


def test_fp64_sigma_check_budget_then_off(torch_dev, orc):
    # FP64 restarts on a sigma mismatch at most 32 times a solve; with a threshold so tight that
    # nearly every step mismatches, the solve still converges (the check is off past the budget)
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 2, grid=W.Grid(40, 60, 30))
    ctx = context([g.shape], env=dict(EQS_SIGMA_TOL=1e-16, EQS_SMALL=0))
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-10, maxit=5000)
    ctx.close()
    assert info["status"] == 0 and info["sigma_restarts"] == 32, info
    assert orc.rel_residual(g.shape, diags, b, host(x)) <= 1e-10


@pytest.mark.parametrize("precision", ["fp32_refine", "fp32"])
def test_refinement_housekeeping_in_stream(torch_dev, orc, precision):
    # The refinement's per-set housekeeping (form the inner iterate, update x, the FP64 residual,
    # f for the next inner solve) either runs in the launch stream after every step, or between
    # chunks when the host sees a set's inner solve end.  Every kernel acts only on the sets whose
    # state asks for it, in the same order, so both give the bits of the sets solved one at a time;
    # the pressure-like sets make the FP32 step restart on sigma mismatches along the way (the
    # symmetric form is off, so that a set solved alone runs the form the mixed batch runs).
    torch, dev = torch_dev
    shapes = [(24, 96, 24), (33, 64, 17), (25, 96, 24), (20, 40, 30)]
    cfgs = [2, 1, 2, 1]
    systems = [manufactured(orc, c, grid=W.Grid(*sh), set_id=i) for i, (c, sh) in enumerate(zip(cfgs, shapes))]
    Ds = [dev_arrays(torch, dev, s_[1]) for s_ in systems]
    bs = [dev_arrays(torch, dev, [s_[2]])[0] for s_ in systems]
    tol = 1e-10 if precision == "fp32_refine" else 1e-5
    out = {}
    for name, env in (("instream", dict(EQS_REFINE_INSTREAM_CELLS=0)), ("rounds", dict(EQS_REFINE_INSTREAM=0)),
                      ("instream_eager", dict(EQS_REFINE_INSTREAM_CELLS=0, EQS_GRAPHS=0))):
        ctx = context(shapes, precision=precision, env=dict(env, EQS_SYM=0))
        xb, infos = ctx.solve_batched(Ds, bs, tol=tol, maxit=4000)
        out[name] = ([host(x) for x in xb], infos)
        if name == "instream":
            for i, s_ in enumerate(systems):
                xi, info = ctx.solve(Ds[i], bs[i], tol=tol, maxit=4000, set_id=i)
                assert np.array_equal(host(xi), out[name][0][i]), i
                assert info == infos[i]
        ctx.close()
    print(precision, [i["sigma_restarts"] for i in out["instream"][1]], [i["iters"] for i in out["instream"][1]], flush=True)
    for i, s_ in enumerate(systems):
        assert out["instream"][1][i]["status"] == 0, out["instream"][1][i]
        assert orc.rel_residual(s_[0].shape, s_[1], s_[2], out["instream"][0][i]) <= tol
        for other in ("rounds", "instream_eager"):
            assert np.array_equal(out["instream"][0][i], out[other][0][i]), (i, other)
            assert out["instream"][1][i] == out[other][1][i], (i, other)


def _batched_full_size(torch, dev, orc, cfg, precisions, env=None):
    """Every set of workload cfg at full size, solved in one batched call to 1e-10 per precision;
    the oracle recomputes each set's residual and bounds its forward error."""
    systems = []
    for i in range(len(W.CONFIGS[cfg]["grids"])):
        systems.append(manufactured(orc, cfg, set_id=i))
        print("config%d set %d generated" % (cfg, i), flush=True)
    grids = [s[0].shape for s in systems]
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    for precision in precisions:
        # "fp64_mg": FP64 with the multigrid preconditioner, all sets iterating together
        ctx = context(grids, precision="fp64" if precision == "fp64_mg" else precision, env=env)
        if precision == "fp64_mg":
            ctx.set_preconditioner("mg", gamma=1.0, coarse_sweeps=15, coarse_cells=2048)
        xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=W.CONFIGS[cfg]["maxit"])
        print("config%d batched %s" % (cfg, precision), infos, flush=True)
        for i, (g, diags, b, xs) in enumerate(systems):
            assert infos[i]["status"] == 0, (precision, i, infos[i])
            xg = host(xb[i])
            assert orc.rel_residual(g.shape, diags, b, xg) <= 1e-10, (precision, i)
            assert np.max(np.abs(xg - xs)) <= orc.forward_error_certificate(g.shape, diags, b, xg) * (1 + 1e-6)
        ctx.close()
        del xb


def test_config2_full_size_batched(torch_dev, orc):
    """The four staggered sets of a time step (96-97 x 384-385 x 96-97), FP64, FP32 + refinement and
    FP64 with the multigrid preconditioner."""
    torch, dev = torch_dev
    _batched_full_size(torch, dev, orc, 2, ["fp64", "fp32_refine", "fp64_mg"])


def test_config4_full_size_batched(torch_dev, orc):
    """The large tall bed: four 192 x 768 x 192 sets (113 M cells) in one call, FP32 + refinement, FP64
    and FP64 with the multigrid preconditioner."""
    torch, dev = torch_dev
    _batched_full_size(torch, dev, orc, 4, ["fp32_refine", "fp64", "fp64_mg"])


# ---------------------------------------------------------------- multigrid preconditioner

MG_SMALL = dict(omega=0.8, gamma=1.6, coarse_sweeps=7, coarse_cells=16)


@pytest.mark.parametrize("cfg,shape", [(0, (20, 17, 9)), (1, (33, 64, 17)), (0, (5, 1, 1)), (2, (1, 40, 3)),
                                       (1, (16, 16, 16))])
def test_mg_vcycle_matches_oracle(torch_dev, orc, cfg, shape):
    # the V-cycle takes the definition's operations in its order with no FMA contraction, on the
    # system's coefficients rounded to FP32 (its level-0 operator): the same bits as the oracle's
    # plain evaluation of the V-cycle of that operator
    from oracle import oracle as O
    torch, dev = torch_dev
    g = W.Grid(*shape)
    diags = W.make_set(cfg, 0, grid=g)["diags"]
    r = np.random.default_rng(11).standard_normal(g.n)
    rounded = [d.astype(np.float32).astype(np.float64) for d in diags]
    zo, lo = orc.mg_apply(g.shape, rounded, r, O.mg_params(**MG_SMALL))
    # coarse levels read as symmetric where they are (the pressure-like recipe) or always in full
    for env in (dict(), dict(EQS_MG_SYM=0), dict(EQS_MG_CSYM=0)):
        old = {k: os.environ.get(k) for k in env}
        os.environ.update({k: str(v) for k, v in env.items()})
        try:
            ctx = context([g.shape])
            ctx.set_preconditioner("mg", **MG_SMALL)
            z, lev = ctx.precond_apply(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [r])[0])
            ctx.close()
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        zg = host(z)
        assert lev == lo
        err = np.max(np.abs(zg - zo)) / np.max(np.abs(zo))
        print("mg vcycle", shape, env, "levels", lev, "bitwise", np.array_equal(zg, zo), "max rel diff %.2e" % err,
              flush=True)
        assert np.array_equal(zg, zo), env


@pytest.mark.parametrize("cfg,shape,gamma", [(1, (32, 64, 32), 1.6), (0, (20, 30, 15), 1.0), (2, (25, 48, 24), 1.0)])
def test_mg_solve_matches_oracle(torch_dev, orc, cfg, shape, gamma):
    from oracle import oracle as O
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, cfg, grid=W.Grid(*shape))
    prm = dict(omega=0.8, gamma=gamma, coarse_sweeps=30, coarse_cells=512)
    xo, oinfo = orc.bicgstab_mg(g.shape, diags, b, tol=1e-12, maxit=500, params=O.mg_params(**prm))
    assert oinfo["status"] == 0
    ctx = context([g.shape])
    ctx.set_preconditioner("mg", **prm)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-12, maxit=500)
    xg = host(x)
    print("mg solve", shape, "gpu", info, "oracle", oinfo, flush=True)
    assert info["status"] == 0
    assert orc.rel_residual(g.shape, diags, b, xg) <= 1e-12
    assert abs(info["iters"] - oinfo["iters"]) <= 2
    assert np.max(np.abs(xg - xs)) <= orc.forward_error_certificate(g.shape, diags, b, xg) * (1 + 1e-6)
    if cfg != 1:  # well-conditioned systems: the two solutions agree to 1e-10
        assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


def test_mg_batched_equals_sequential_and_statuses(torch_dev, orc):
    torch, dev = torch_dev
    systems = [manufactured(orc, 2, grid=W.Grid(*s), set_id=i) for i, s in enumerate(STAGGERED_SMALL)]
    ctx = context(STAGGERED_SMALL)
    ctx.set_preconditioner("mg")
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=500)
    for i, s in enumerate(systems):
        xi, info = ctx.solve(Ds[i], bs[i], tol=1e-10, maxit=500, set_id=i)
        assert np.array_equal(host(xi), host(xb[i])) and info == infos[i]
        assert orc.rel_residual(s[0].shape, s[1], s[2], host(xb[i])) <= 1e-10
    # maxit too small: computed, not converged; exact initial guess: no iteration; b = 0: x = 0
    g, diags, b, xs = systems[0]
    x, info = ctx.solve(Ds[0], bs[0], tol=1e-13, maxit=1, check=False)
    assert info["status"] == 1 and info["iters"] == 1
    assert abs(info["rel_res"] - orc.rel_residual(g.shape, diags, b, host(x))) <= 1e-8 * info["rel_res"]
    x, info = ctx.solve(Ds[0], bs[0], x=dev_arrays(torch, dev, [xs])[0], tol=1e-10)
    assert info["iters"] == 0 and np.array_equal(host(x), xs)
    x, info = ctx.solve(Ds[0], torch.zeros_like(bs[0]), x=torch.ones_like(bs[0]), tol=1e-10)
    assert info["status"] == 0 and not np.any(host(x))


def test_mg_batched_mixed_depths(torch_dev, orc):
    # sets of different hierarchy depths in one batched multigrid call (4 levels, 1 level -- the
    # whole set is the coarsest level --, 3 levels, 2 levels): each set follows its own V-cycle, the
    # same bits as solved alone and as the oracle's V-cycle iteration count
    from oracle import oracle as O
    torch, dev = torch_dev
    shapes = [(40, 40, 40), (8, 8, 8), (17, 9, 30), (12, 10, 6)]
    systems = [manufactured(orc, 2, grid=W.Grid(*sh), set_id=i) for i, sh in enumerate(shapes)]
    prm = dict(omega=0.8, gamma=1.0, coarse_sweeps=30, coarse_cells=512)
    ctx = context(shapes)
    ctx.set_preconditioner("mg", **prm)
    Ds = [dev_arrays(torch, dev, s_[1]) for s_ in systems]
    bs = [dev_arrays(torch, dev, [s_[2]])[0] for s_ in systems]
    xb, infos = ctx.solve_batched(Ds, bs, tol=1e-11, maxit=500)
    for i, s_ in enumerate(systems):
        xi, info = ctx.solve(Ds[i], bs[i], tol=1e-11, maxit=500, set_id=i)
        assert np.array_equal(host(xi), host(xb[i])) and info == infos[i], i
        assert orc.rel_residual(s_[0].shape, s_[1], s_[2], host(xb[i])) <= 1e-11
        _, oinfo = orc.bicgstab_mg(s_[0].shape, s_[1], s_[2], tol=1e-11, maxit=500, params=O.mg_params(**prm))
        assert abs(infos[i]["iters"] - oinfo["iters"]) <= 2, (i, infos[i], oinfo)
    ctx.close()


@pytest.mark.parametrize("cfg,shape", [(0, (20, 30, 15)), (1, (32, 64, 32)), (2, (25, 48, 24))])
def test_mg_adjoint_matches_oracle(torch_dev, orc, cfg, shape):
    # With multigrid selected the adjoint solves A^T lambda = w with the V-cycle of A^T: lambda
    # meets tol in the oracle's transposed residual, takes the oracle's multigrid iteration count
    # on A^T's rows (formed here independently from the definition), and the gradients equal the
    # oracle's from its own Jacobi adjoint
    from oracle import oracle as O
    torch, dev = torch_dev
    g = W.Grid(*shape)
    s_ = W.make_set(cfg, 0, grid=g, with_weights=True)
    diags, w = s_["diags"], s_["w"]
    b = orc.apply(g.shape, diags, s_["x_star"])
    xo, _ = orc.bicgstab(g.shape, diags, b, tol=1e-13, maxit=5000)
    lo, linfo = orc.bicgstab(g.shape, diags, w, tol=1e-13, maxit=5000, transpose=True)
    assert linfo["status"] == 0
    Go = orc.grad(g.shape, lo, xo)
    # rows of A^T: a_P, and the links of the neighbours pointing at the cell
    nx, ny, nz = g.nx, g.ny, g.nz
    a = [d.reshape(nz, ny, nx) for d in diags]
    at = [a[0].copy()] + [np.zeros_like(a[0]) for _ in range(6)]
    at[1][:, :, :-1] = a[2][:, :, 1:]    # E^T(c) = W(c+1)
    at[2][:, :, 1:] = a[1][:, :, :-1]    # W^T(c) = E(c-1)
    at[3][:, :-1, :] = a[4][:, 1:, :]    # N^T(c) = S(c+nx)
    at[4][:, 1:, :] = a[3][:, :-1, :]    # S^T(c) = N(c-nx)
    at[5][:-1, :, :] = a[6][1:, :, :]    # T^T(c) = B(c+P)
    at[6][1:, :, :] = a[5][:-1, :, :]    # B^T(c) = T(c-P)
    at = [x.ravel() for x in at]
    prm = dict(omega=0.8, gamma=1.6 if cfg == 1 else 1.0, coarse_sweeps=30, coarse_cells=512)
    lm, minfo = orc.bicgstab_mg(g.shape, at, w, tol=1e-12, maxit=500, params=O.mg_params(**prm))
    assert minfo["status"] == 0
    ctx = context([g.shape])
    ctx.set_preconditioner("mg", **prm)
    D = dev_arrays(torch, dev, diags)
    xd, wd = dev_arrays(torch, dev, [xo, w])
    gb, gd, info = ctx.adjoint(D, xd, wd, tol=1e-12, maxit=500)
    gb2, _, info2 = ctx.adjoint(D, xd, wd, tol=1e-12, maxit=500)   # again, in the same context
    ctx.close()
    print("mg adjoint", cfg, shape, info, "oracle mg on A^T", minfo["iters"], "jacobi", linfo["iters"], flush=True)
    assert np.array_equal(host(gb), host(gb2)) and info == info2
    assert info["status"] == 0
    assert orc.rel_residual(g.shape, diags, w, host(gb), transpose=True) <= 1e-12
    assert abs(info["iters"] - minfo["iters"]) <= 2
    if cfg != 1:
        assert np.linalg.norm(host(gb) - lo) <= 1e-9 * np.linalg.norm(lo)
        for k in range(7):
            assert np.linalg.norm(host(gd[k]) - Go[k]) <= 1e-9 * np.linalg.norm(Go[k]) + 1e-300, k
    else:  # near-singular: the solutions agree to what the residual bound allows
        assert np.linalg.norm(host(gb) - lo) <= 1e-6 * np.linalg.norm(lo)


def test_mg_needs_an_fp64_context(torch_dev):
    from paper_2211_15605_amd.solver import EqSolveError
    ctx = context([(8, 8, 8)], precision="fp32_refine")
    with pytest.raises(EqSolveError):
        ctx.set_preconditioner("mg")
    ctx = context([(8, 8, 8)])
    with pytest.raises(EqSolveError):
        ctx.set_preconditioner("mg", coarse_cells=4096)  # beyond the one-block coarsest solve


def test_mg_config1_full_size(torch_dev, orc):
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1)
    ctx = context([g.shape])
    ctx.set_preconditioner("mg", gamma=1.6)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-10, maxit=500)
    print("config1 mg", info, flush=True)
    assert info["status"] == 0 and info["iters"] <= 40
    xg = host(x)
    assert orc.rel_residual(g.shape, diags, b, xg) <= 1e-10
    assert np.max(np.abs(xg - xs)) <= orc.forward_error_certificate(g.shape, diags, b, xg) * (1 + 1e-6)


def _mg_solve_with_sym(torch, dev, g, diags, b, sym_env):
    old = os.environ.get("EQS_MG_SYM")
    os.environ["EQS_MG_SYM"] = sym_env
    try:
        ctx = context([g.shape])
        ctx.set_preconditioner("mg", gamma=1.6, coarse_cells=64)
        x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-11, maxit=500)
        return host(x), info
    finally:
        if old is None:
            os.environ.pop("EQS_MG_SYM", None)
        else:
            os.environ["EQS_MG_SYM"] = old


def test_mg_symmetric_reads_are_exact_and_detected(torch_dev, orc):
    """An exactly symmetric matrix (the pressure-like recipe) lets the multigrid iteration read
    a_W, a_S, a_B as a_E, a_N, a_T of the neighbour: the same values, so the same bits as with that
    off.  One perturbed coefficient makes the matrix non-symmetric: the check must see it (else the
    iteration would run on another operator and the true residual would not meet tol)."""
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1, grid=W.Grid(24, 40, 20))
    x1, i1 = _mg_solve_with_sym(torch, dev, g, diags, b, "1")
    x0, i0 = _mg_solve_with_sym(torch, dev, g, diags, b, "0")
    assert i1 == i0 and np.array_equal(x1, x0)
    assert orc.rel_residual(g.shape, diags, b, x1) <= 1e-11
    pert = [d.copy() for d in diags]
    c = 5 + g.nx * (7 + g.ny * 9)           # an interior cell
    pert[2][c] *= 1.001                     # a_W(c) != a_E(c - 1)
    bp = orc.apply(g.shape, pert, xs)
    x1, i1 = _mg_solve_with_sym(torch, dev, g, pert, bp, "1")
    x0, i0 = _mg_solve_with_sym(torch, dev, g, pert, bp, "0")
    assert i1["status"] == 0 and i1 == i0 and np.array_equal(x1, x0)
    assert orc.rel_residual(g.shape, pert, bp, x1) <= 1e-11


def test_preconditioner_switch_restores_the_jacobi_tiling(torch_dev, orc):
    """Selecting multigrid re-tiles the sets (fewer planes per chunk for its fine-level passes);
    going back to Jacobi restores the Jacobi iteration's own tiling, so its solves repeat bit for
    bit (same tiles, same reduction order)."""
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1, grid=W.Grid(40, 64, 48))
    ctx = context([g.shape], env=dict(EQS_KC=16))
    D = dev_arrays(torch, dev, diags)
    bd = dev_arrays(torch, dev, [b])[0]
    lay0 = ctx.layout()
    x0, i0 = ctx.solve(D, bd, tol=1e-10, maxit=2000)
    ctx.set_preconditioner("mg")
    lay_mg = ctx.layout()
    assert lay_mg["kc"] == 8 and lay_mg["cpt"] == lay0["cpt"], (lay0, lay_mg)
    xm, im = ctx.solve(D, bd, tol=1e-10, maxit=500)
    assert orc.rel_residual(g.shape, diags, b, host(xm)) <= 1e-10
    ctx.set_preconditioner("jacobi")
    assert ctx.layout()["kc"] == lay0["kc"] == 16
    x1, i1 = ctx.solve(D, bd, tol=1e-10, maxit=2000)
    assert i1 == i0 and np.array_equal(host(x1), host(x0))


# ---------------------------------------------------------------- symmetric form of the single-sync step
#
# An exactly symmetric matrix (the pressure-like recipe) lets the single-sync step form the products
# of A D^-1 from a_E, a_N, a_T and 1/a_P: the same operator, evaluated with other roundings.  The
# form is reported in info["symmetric"]; EQS_SYM=0 turns it off.

SYM_SHAPES = [(33, 64, 17), (130, 3, 40), (200, 7, 3), (97, 31, 5), (1, 300, 2), (3, 1, 700), (60, 45, 1)]


def _sym_solve(torch, dev, g, diags, b, precision="fp64", env=None, tol=1e-12, maxit=20000):
    ctx = context([g.shape], precision=precision, env=dict(env or {}, EQS_SMALL=0))
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=tol, maxit=maxit)
    ctx.close()
    return host(x), info


@pytest.mark.parametrize("shape", SYM_SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "fp32"])
def test_symmetric_form_meets_tol_against_oracle(torch_dev, orc, shape, precision):
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1, grid=W.Grid(*shape))
    tol = {"fp64": 1e-12, "fp32_refine": 1e-10, "fp32": 1e-5}[precision]
    for env, sym in ((dict(), True), (dict(EQS_SYM=0), False)):
        xg, info = _sym_solve(torch, dev, g, diags, b, precision, env, tol=tol)
        print(shape, precision, env, info, flush=True)
        assert info["status"] == 0 and info["symmetric"] is sym, (env, info)
        rel = orc.rel_residual(g.shape, diags, b, xg)
        assert rel <= tol, (env, rel)
        assert abs(rel - info["rel_res"]) <= 1e-3 * rel
        assert np.max(np.abs(xg - xs)) <= orc.forward_error_certificate(g.shape, diags, b, xg) * (1 + 1e-6)


@pytest.mark.parametrize("tiling", TILINGS[1:] + [dict(EQS_SMALL=0, EQS_CPT=1, EQS_KC=5)] +
                         [dict(f, EQS_SMALL=0) for f in FUSED_SHAPES],
                         ids=["cpt1_kc1", "cpt2_kc3", "cpt2_kc7", "cpt1_kc5"] + FUSED_IDS)
def test_symmetric_form_launch_layouts(torch_dev, orc, tiling):
    """Every tile layout (cells per thread, planes per chunk, halo slots) of the symmetric form
    against the oracle's FP64 residual, and against the general form's solution."""
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1, grid=W.Grid(37, 23, 19))
    xo, oinfo = orc.bicgstab(g.shape, diags, b, tol=1e-13, maxit=20000)
    assert oinfo["status"] == 0
    xs1, i1 = _sym_solve(torch, dev, g, diags, b, env=tiling, tol=1e-13)
    xg0, i0 = _sym_solve(torch, dev, g, diags, b, env=dict(tiling, EQS_SYM=0), tol=1e-13)
    assert i1["symmetric"] and not i0["symmetric"]
    for xg in (xs1, xg0):
        assert orc.rel_residual(g.shape, diags, b, xg) <= 1e-13
        cert = orc.forward_error_certificate(g.shape, diags, b, xg)
        assert np.max(np.abs(xg - xo)) <= 2 * cert + orc.forward_error_certificate(g.shape, diags, b, xo)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_symmetric_form_detection_is_exact(torch_dev, orc, precision):
    """The check (in the scale pass, or the cast pass of the FP32 forms) compares the stored values
    bit for bit: one a_W one ulp off its partner a_E makes the matrix non-symmetric (the general
    form, the same bits as with the form off), while coefficients pointing out of the grid, which
    no product uses, do not count."""
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1, grid=W.Grid(24, 40, 20))
    pert = [d.copy() for d in diags]
    c = 5 + g.nx * (7 + g.ny * 9)
    pert[2][c] = np.nextafter(pert[2][c], np.inf)  # a_W(c) != a_E(c - 1) by one ulp
    bp = orc.apply(g.shape, pert, xs)
    x1, i1 = _sym_solve(torch, dev, g, pert, bp, precision, tol=1e-11)
    x0, i0 = _sym_solve(torch, dev, g, pert, bp, precision, env=dict(EQS_SYM=0), tol=1e-11)
    assert not i1["symmetric"] and i1 == i0 and np.array_equal(x1, x0)
    assert orc.rel_residual(g.shape, pert, bp, x1) <= 1e-11
    # nonzero links out of the grid (a_W at i = 0, a_N at j = ny-1, a_B at k = 0): still symmetric,
    # and the solution does not see them
    outw = [d.copy() for d in diags]
    rng = np.random.default_rng(7)
    idx = np.arange(g.n).reshape(g.nz, g.ny, g.nx)
    for arr, sel in ((2, idx[:, :, 0]), (3, idx[:, -1, :]), (6, idx[0, :, :])):
        outw[arr][sel.ravel()] = rng.uniform(0.5, 2.0, sel.size)
    x2, i2 = _sym_solve(torch, dev, g, outw, b, precision, tol=1e-11)
    assert i2["symmetric"] and i2["status"] == 0
    xr, ir = _sym_solve(torch, dev, g, diags, b, precision, tol=1e-11)
    assert ir["symmetric"] and i2 == ir and np.array_equal(x2, xr)


def test_symmetric_form_batched_and_graphs(torch_dev, orc):
    """A batched call takes the form only when every set is symmetric; then each set equals its own
    solve bit for bit, and graph replays equal eager launches.  A mixed batch runs the general form
    for all of its sets (the same bits as with the form off)."""
    torch, dev = torch_dev
    shapes = [(24, 96, 24), (25, 96, 24)]
    sym = [manufactured(orc, 1, grid=W.Grid(*s), set_id=i) for i, s in enumerate(shapes)]
    cd = manufactured(orc, 2, grid=W.Grid(*shapes[1]), set_id=1)
    for systems, want in ((sym, True), ([sym[0], cd], False)):
        Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
        bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
        ctx = context(shapes)
        xb, infos = ctx.solve_batched(Ds, bs, tol=1e-11, maxit=3000)
        for i, s in enumerate(systems):
            assert infos[i]["status"] == 0 and infos[i]["symmetric"] is want, (i, infos[i])
            assert orc.rel_residual(s[0].shape, s[1], s[2], host(xb[i])) <= 1e-11
        if want:
            for i in range(2):
                xi, info = ctx.solve(Ds[i], bs[i], tol=1e-11, maxit=3000, set_id=i)
                assert np.array_equal(host(xi), host(xb[i])) and info == infos[i], i
            eager = context(shapes, env=dict(EQS_GRAPHS=0))
            xe, ie = eager.solve_batched(Ds, bs, tol=1e-11, maxit=3000)
            for rep in range(3):
                junk = torch.randn(1 << 20, device=dev, dtype=torch.float64).cumsum(0)
                torch.cuda.synchronize()
                xr, ir = ctx.solve_batched(Ds, bs, tol=1e-11, maxit=3000)
                assert ir == ie and all(np.array_equal(host(a), host(e)) for a, e in zip(xr, xe)), rep
                del junk
            eager.close()
        else:
            off = context(shapes, env=dict(EQS_SYM=0))
            xo, io = off.solve_batched(Ds, bs, tol=1e-11, maxit=3000)
            assert io == infos and all(np.array_equal(host(a), host(e)) for a, e in zip(xb, xo))
            off.close()
        ctx.close()


def test_symmetric_matrix_adjoint_runs_the_transposed_general_form(torch_dev, orc):
    """The adjoint iterates on A^T D^-1 through the transposed scale pass; it never takes the
    symmetric form (reported clear), and on a symmetric matrix lambda = A^-T w equals the forward
    solve with w as right-hand side to the solves' tolerance."""
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 1, grid=W.Grid(20, 24, 16))
    D = dev_arrays(torch, dev, diags)
    ctx = context([g.shape], env=dict(EQS_SMALL=0))
    x, fi = ctx.solve(D, dev_arrays(torch, dev, [b])[0], tol=1e-13, maxit=5000)
    assert fi["symmetric"] and fi["status"] == 0
    w = np.random.default_rng(5).standard_normal(g.n)
    gb, gd, ai = ctx.adjoint(D, x, dev_arrays(torch, dev, [w])[0], tol=1e-13, maxit=5000)
    assert ai["status"] == 0 and not ai["symmetric"], ai
    lam = host(gb)
    assert orc.rel_residual(g.shape, diags, w, lam) <= 1e-12  # A^T = A: lambda solves A lambda = w
    xw, wi = ctx.solve(D, dev_arrays(torch, dev, [w])[0], tol=1e-13, maxit=5000)
    cert = orc.forward_error_certificate(g.shape, diags, w, lam) + orc.forward_error_certificate(g.shape, diags, w, host(xw))
    assert np.max(np.abs(lam - host(xw))) <= cert * (1 + 1e-6)


# ---------------------------------------------------------------- wide rows

# with the single-sync step's LDS capped at 64 KB, rows of 203..266 cells take it with one cell per
# thread (257..266 with four halo slots per ring) and wider rows the three-launch iteration; with
# the device's 160 KB, two cells per thread up to 512 (257..512: four halo slots); wider rows, up to
# the largest the library takes (1024), run the three-launch iteration with eight halo slots
WIDE = [(230, 5, 4), (260, 5, 4), (266, 3, 3), (400, 4, 3), (700, 3, 4), (1024, 3, 3)]


@pytest.mark.parametrize("shape", WIDE)
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("scheme", SCHEMES + [dict(EQS_FNT=512), dict(EQS_FUSED_LDS=65536)],
                         ids=SCHEME_IDS + ["fnt512", "lds64k"])
def test_wide_rows_against_oracle(torch_dev, orc, shape, precision, scheme):
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 0, grid=W.Grid(*shape))
    tol = 1e-13 if precision == "fp64" else 1e-10
    ctx = context([g.shape], precision=precision, env=scheme)
    lay = ctx.layout()
    print("wide", shape, precision, scheme, lay, flush=True)
    x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=tol, maxit=5000)
    ctx.close()
    assert info["status"] == 0, info
    xg = host(x)
    assert orc.rel_residual(g.shape, diags, b, xg) <= tol
    if precision == "fp64":
        xo, _ = orc.bicgstab(g.shape, diags, b, tol=1e-13, maxit=5000)
        assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


# ---------------------------------------------------------------- adjoint against finite differences

def test_adjoint_config3_central_finite_differences(torch_dev, orc):
    # The adjoint workload (64^3 convection-diffusion, L = sum(w x)): the gradients the GPU adjoint
    # returns for b and the 7 diagonals, against central differences of GPU forward solves with
    # h = 1e-6 along sparse Rademacher directions.  The perturbed solves start from the converged x
    # and run to 1e-15 (or until they stagnate), so the FD quotient is limited by h^2 and by the
    # solves' rounding, far below 1e-5.
    torch, dev = torch_dev
    import math
    g = W.Grid(64, 64, 64)
    s = W.make_set(3, 0, grid=g, with_weights=True)
    diags, w = s["diags"], s["w"]
    b = orc.apply(g.shape, diags, s["x_star"])
    ctx = context([g.shape])
    D = dev_arrays(torch, dev, diags)
    bd, wd = dev_arrays(torch, dev, [b, w])
    x, info = ctx.solve(D, bd, tol=1e-15, maxit=3000, check=False)
    assert info["rel_res"] <= 1e-14, info
    gb, gd, ainfo = ctx.adjoint(D, x, wd, tol=1e-14, maxit=3000, check=False)
    assert ainfo["rel_res"] <= 1e-13, ainfo
    G = [host(gb)] + [host(t) for t in gd]   # dL/db, then P, E, W, N, S, T, B
    h = 1e-6
    rng = np.random.default_rng(2211)
    base = [bd] + D
    for direction in range(6):
        # 8192 entries spread over the 8 arrays (b and the diagonals; 0.4 % of their 2.1 M
        # entries), signs +-1: enough signal that the solves' rounding floor stays far below 1e-5
        m = 8192
        arr = rng.integers(0, 8, m)
        idx = rng.integers(0, g.n, m)
        sgn = rng.choice([-1.0, 1.0], m)
        delta = [np.zeros(g.n) for _ in range(8)]
        for a in range(8):
            np.add.at(delta[a], idx[arr == a], h * sgn[arr == a])
        dd = dev_arrays(torch, dev, delta)
        plus = [t + e for t, e in zip(base, dd)]
        minus = [t - e for t, e in zip(base, dd)]
        # first-order change predicted by the adjoint, for the perturbation actually applied
        pred = math.fsum(math.fsum((G[a] * host(plus[a] - minus[a])).tolist()) for a in range(8))
        xp, ip = ctx.solve(plus[1:], plus[0], x.clone(), tol=1e-15, maxit=3000, check=False)
        xm, im = ctx.solve(minus[1:], minus[0], x.clone(), tol=1e-15, maxit=3000, check=False)
        assert ip["rel_res"] <= 1e-14 and im["rel_res"] <= 1e-14, (ip, im)
        fd = math.fsum((w * (host(xp) - host(xm))).tolist())
        print("direction %d: FD %.12e adjoint %.12e rel %.2e (%d, %d iterations)" % (
            direction, fd, pred, abs(fd - pred) / abs(pred), ip["iters"], im["iters"]), flush=True)
        assert abs(fd - pred) <= 1e-5 * abs(pred)
    ctx.close()


def test_fused_launch_shapes_are_taken(torch_dev, orc):
    # the environment selects the single-sync step's block size and tile order, and the layout
    # reports what runs: 512 threads over 1024-cell segments where the shape allows it
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, 2, grid=W.Grid(96, 40, 9))
    lay = {}
    for name, env in (("default", dict()), ("fnt512", dict(EQS_FNT=512)), ("ford1", dict(EQS_FORD=1))):
        ctx = context([g.shape], env=env)
        x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-12, maxit=3000)
        lay[name] = ctx.layout()
        ctx.close()
        assert info["status"] == 0 and orc.rel_residual(g.shape, diags, b, host(x)) <= 1e-12, name
    assert lay["default"]["fused_threads"] == 256 and lay["default"]["fused_order"] == 0
    assert lay["fnt512"]["fused_threads"] == 512 and lay["fnt512"]["fused_segments"] == (96 * 40 + 1023) // 1024
    assert lay["fnt512"]["fused_tiles"] == lay["fnt512"]["fused_segments"] * lay["fnt512"]["chunks"]
    assert lay["ford1"]["fused_order"] == 1


# ---------------------------------------------------------------- unscaled form of the step

@pytest.mark.parametrize("cfg,shape", [(0, (16, 16, 16)), (0, (33, 17, 9)), (2, (97, 31, 5)), (0, (200, 7, 3)),
                                       (1, (37, 23, 19)), (0, (1, 300, 2))])
def test_unscaled_form_matches_oracle(torch_dev, orc, cfg, shape):
    # the single-sync step from the caller's coefficients and 1/a_P (no scale pass), in several
    # launch shapes, against the oracle's solution; a symmetric system runs it too (the symmetric
    # form is not used: its check belongs to the scale pass)
    torch, dev = torch_dev
    g, diags, b, xs = manufactured(orc, cfg, grid=W.Grid(*shape))
    xo, oinfo = orc.bicgstab(g.shape, diags, b, tol=1e-13, maxit=20000)
    assert oinfo["status"] == 0
    for env in (dict(EQS_SMALL=0), dict(EQS_SMALL=0, EQS_FNT=512), dict(EQS_SMALL=0, EQS_FORD=1, EQS_KC=3)):
        ctx = context([g.shape], env=env)
        ctx.set_step_form("unscaled")
        x, info = ctx.solve(dev_arrays(torch, dev, diags), dev_arrays(torch, dev, [b])[0], tol=1e-13, maxit=20000)
        ctx.close()
        xg = host(x)
        assert info["status"] == 0 and info["unscaled"] and not info["symmetric"], (env, info)
        assert orc.rel_residual(g.shape, diags, b, xg) <= 1e-13
        if cfg != 1:
            assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo), env
        else:   # near-singular: bounded by the certificates of both solutions
            cert = orc.forward_error_certificate(g.shape, diags, b, xg)
            assert np.max(np.abs(xg - xo)) <= 2 * cert + orc.forward_error_certificate(g.shape, diags, b, xo)


def test_unscaled_form_batched_equals_sequential_and_graphs(torch_dev, orc):
    torch, dev = torch_dev
    systems = [manufactured(orc, 2, grid=W.Grid(*s), set_id=i) for i, s in enumerate(STAGGERED_SMALL)]
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    out = []
    for env in (dict(), dict(EQS_GRAPHS=0)):
        ctx = context(STAGGERED_SMALL, env=env)
        ctx.set_step_form("unscaled")
        xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=2000)
        for i, s in enumerate(systems):
            xi, info = ctx.solve(Ds[i], bs[i], tol=1e-10, maxit=2000, set_id=i)
            assert np.array_equal(host(xi), host(xb[i])), i
            assert info == infos[i] and info["unscaled"]
            assert orc.rel_residual(s[0].shape, s[1], s[2], host(xb[i])) <= 1e-10
        out.append([host(x) for x in xb])
        ctx.close()
    assert all(np.array_equal(a, b) for a, b in zip(out[0], out[1]))   # graph replay == eager


def test_step_form_is_for_fp64_contexts(torch_dev):
    from paper_2211_15605_amd.solver import EqSolveError
    ctx = context([(8, 8, 8)], precision="fp32_refine")
    with pytest.raises(EqSolveError):
        ctx.set_step_form("unscaled")
    ctx.close()


@pytest.mark.parametrize("nreads,nt", [(13, 1), (11, 1), (13, 0)])
def test_stream_probe_writes_its_definition(torch_dev, nreads, nt):
    # the streaming kernel the step's rate is read against: out_w = w + sum_k (k+1) in_k on every
    # cell, a ragged count (not a multiple of the 512 cells of a block), nothing written past n
    torch, dev = torch_dev
    from paper_2211_15605_amd import binding
    n = 5 * 512 + 77
    rng = np.random.default_rng(11)
    ins = [torch.from_numpy(rng.uniform(-1, 1, n)).to(dev) for _ in range(nreads)]
    outs = [torch.full((n + 64,), 7.0, dtype=torch.float64, device=dev) for _ in range(5)]
    rc = binding.eqsolve_debug_stream([t.data_ptr() for t in ins], [t.data_ptr() for t in outs], n, nt,
                                      torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    s = np.zeros(n)
    for k in range(nreads):
        s = s + (k + 1) * host(ins[k])
    for w in range(5):
        o = host(outs[w])
        assert np.allclose(o[:n], s + w, rtol=0, atol=64 * EPS * np.max(np.abs(s) + w))
        assert np.all(o[n:] == 7.0)


# ---------------------------------------------------------------- XCD-balanced block map

# each XCD runs a share of every set of a batched launch; the shapes give tile, step-tile and
# pointwise-block counts that are multiples of 8 (64 x 64 planes in 512-cell segments, 8-plane
# chunks, 64 pointwise blocks) and counts that are not (the ragged grids)
XBAL_CASES = {
    "mult8": ([(64, 64, 32), (64, 64, 16), (64, 64, 24)],
              dict(EQS_CPT=2, EQS_KC=8, EQS_FNT=256, EQS_FORD=1, EQS_FLAT_MAX=64, EQS_SMALL=0)),
    "ragged": ([(33, 17, 9), (40, 24, 13), (20, 31, 7), (9, 50, 11)], dict(EQS_KC=3, EQS_SMALL=0)),
}


@pytest.mark.parametrize("case", ["mult8", "ragged"])
@pytest.mark.parametrize("precision,mg", [("fp64", False), ("fp32_refine", False), ("fp64", True)],
                         ids=["fp64", "fp32_refine_instream", "fp64_multigrid"])
def test_xcd_balanced_map_equals_contiguous_map(torch_dev, orc, monkeypatch, case, precision, mg):
    # the block -> (set, tile) map decides only which XCD runs a tile: batched solves under the
    # balanced map equal those under the contiguous one and each set's own solve, bit for bit (FP32:
    # with the refinement's housekeeping launched after every step, which acts on some sets only)
    torch, dev = torch_dev
    shapes, env = XBAL_CASES[case]
    systems = [manufactured(orc, 1 if mg else 2, grid=W.Grid(*sh), set_id=i) for i, sh in enumerate(shapes)]
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    monkeypatch.setenv("EQS_REFINE_INSTREAM_CELLS", "0")
    out = {}
    for xbal in ("1", "0"):
        monkeypatch.setenv("EQS_XBAL", xbal)
        ctx = context(shapes, precision=precision, env=env)
        if mg:
            ctx.set_preconditioner("mg", gamma=1.6, coarse_sweeps=15)
        print("xbal", xbal, case, precision, mg, [ctx.layout(i) for i in range(len(shapes))], flush=True)
        xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=5000)
        out[xbal] = ([host(x) for x in xb], infos)
        if xbal == "1":
            for i in range(len(systems)):
                xi, info = ctx.solve(Ds[i], bs[i], tol=1e-10, maxit=5000, set_id=i)
                assert np.array_equal(host(xi), host(xb[i])) and info == infos[i], i
        ctx.close()
    for i, s in enumerate(systems):
        assert np.array_equal(out["1"][0][i], out["0"][0][i]) and out["1"][1][i] == out["0"][1][i], i
        assert out["1"][1][i]["status"] == 0
        assert orc.rel_residual(s[0].shape, s[1], s[2], out["1"][0][i]) <= 1e-10


def test_eight_sets_batched_equal_their_own_solves(torch_dev, orc):
    # the largest batch a context takes: eight sets of mixed sizes (two of them single-tile, the others
    # ragged multi-tile grids; the one-block solve off, so a set takes the same path alone as in the
    # batch), FP64 and FP32 + refinement, each equal to its own solve bit for bit; a ninth set is refused
    torch, dev = torch_dev
    shapes = [(33, 17, 9), (8, 16, 8), (40, 24, 13), (20, 31, 7), (9, 50, 11), (12, 12, 12), (64, 20, 10),
              (17, 33, 19)]
    systems = [manufactured(orc, 2, grid=W.Grid(*sh), set_id=i % 4) for i, sh in enumerate(shapes)]
    Ds = [dev_arrays(torch, dev, s[1]) for s in systems]
    bs = [dev_arrays(torch, dev, [s[2]])[0] for s in systems]
    for precision in ("fp64", "fp32_refine"):
        ctx = context(shapes, precision=precision, env=dict(EQS_KC=3, EQS_SMALL=0))
        xb, infos = ctx.solve_batched(Ds, bs, tol=1e-10, maxit=5000)
        for i, s in enumerate(systems):
            xi, info = ctx.solve(Ds[i], bs[i], tol=1e-10, maxit=5000, set_id=i)
            assert np.array_equal(host(xi), host(xb[i])) and info == infos[i], (precision, i)
            assert infos[i]["status"] == 0 and orc.rel_residual(s[0].shape, s[1], s[2], host(xb[i])) <= 1e-10
        ctx.close()
    from paper_2211_15605_amd.solver import EqSolveError
    with pytest.raises((EqSolveError, ValueError)):
        context(shapes + [(8, 8, 8)])
