"""eqsolve_solve_noalloc (the FP64 solve on the library's static device workspace) against
eqsolve_solve on a context, through the C ABI: the same kernels and tiles, so the same bits.

Two calls in a row on one GPU, the second on a smaller system, so the second call runs on what
the first left in the shared array.  Also checked by the oracle: residual <= tol in FP64.
"""
import numpy as np
import pytest

from paper_2211_15605_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2211_15605_amd import binding
    binding.load()
    return torch, torch.device("cuda", 0)


def _system(torch, dev, orc, cfg, grid, seed_set):
    s = W.make_set(cfg, seed_set, grid=grid)
    b = orc.apply(grid.shape, s["diags"], s["x_star"])
    D = [torch.from_numpy(d).to(dev) for d in s["diags"]]
    return s, D, torch.from_numpy(b).to(dev), b


def _solve_both(torch, dev, orc, cfg, grid, seed_set, tol, maxit):
    from paper_2211_15605_amd import binding as B
    from paper_2211_15605_amd.solver import Context
    s, D, b, bh = _system(torch, dev, orc, cfg, grid, seed_set)
    print("noalloc: cfg %d grid %s tol %g" % (cfg, grid.shape, tol), flush=True)
    x_na = torch.full_like(b, 0.25)   # the same nonzero x0 for both calls
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc, info = B.eqsolve_solve_noalloc(grid.shape, [d.data_ptr() for d in D], b.data_ptr(), x_na.data_ptr(), tol,
                                       maxit, stream)
    info = info.as_dict()
    with Context([grid.shape], precision="fp64") as ctx:
        x_cx = torch.full_like(b, 0.25)
        rc2, info2 = B.eqsolve_solve(ctx.h, 0, [d.data_ptr() for d in D], b.data_ptr(), x_cx.data_ptr(), tol, maxit)
        info2 = info2.as_dict()
    torch.cuda.synchronize()
    xa, xc = x_na.cpu().numpy(), x_cx.cpu().numpy()
    rel = orc.rel_residual(grid.shape, s["diags"], bh, xa)
    return rc, info, rc2, info2, xa, xc, rel


@pytest.mark.parametrize("first,second", [
    ((0, (40, 24, 20)), (0, (16, 16, 16))),
    ((1, (48, 40, 24)), (0, (30, 9, 7))),
])
def test_noalloc_equals_context_solve_two_calls(torch_dev, orc, first, second):
    torch, dev = torch_dev
    for k, (cfg, shape) in enumerate((first, second)):
        grid = W.Grid(*shape)
        rc, info, rc2, info2, xa, xc, rel = _solve_both(torch, dev, orc, cfg, grid, k, 1e-10, 5000)
        assert rc == 0 and rc2 == 0, (rc, rc2, info, info2)
        assert info["iters"] == info2["iters"] and info["status"] == info2["status"]
        assert np.array_equal(xa, xc), float(np.max(np.abs(xa - xc)))
        assert rel <= 1e-10


def test_noalloc_tiny_system_and_size_limit(torch_dev, orc):
    # a set of <= 2048 cells takes the one-block persistent solve; then a system one plane
    # beyond the limit is refused before any work, with x untouched
    torch, dev = torch_dev
    grid = W.Grid(9, 7, 5)
    rc, info, rc2, info2, xa, xc, rel = _solve_both(torch, dev, orc, 0, grid, 3, 1e-10, 1000)
    assert rc == 0 and rc2 == 0 and np.array_equal(xa, xc) and rel <= 1e-10
    from paper_2211_15605_amd import binding as B
    big = (64, 64, 65)
    n = 64 * 64 * 65
    D = [torch.ones(n, dtype=torch.float64, device=dev) for _ in range(7)]
    b = torch.ones(n, dtype=torch.float64, device=dev)
    x = torch.full_like(b, 3.0)
    rc, _ = B.eqsolve_solve_noalloc(big, [d.data_ptr() for d in D], b.data_ptr(), x.data_ptr(), 1e-10, 10,
                                    torch.cuda.current_stream(dev).cuda_stream)
    assert rc == B.EQS_ERR_SIZE
    assert bool(torch.all(x == 3.0))


def test_noalloc_largest_system(torch_dev, orc):
    # the largest system the static workspace takes (64^3 = EQS_NOALLOC_MAX_CELLS cells)
    torch, dev = torch_dev
    grid = W.Grid(64, 64, 64)
    rc, info, rc2, info2, xa, xc, rel = _solve_both(torch, dev, orc, 3, grid, 0, 1e-10, 1000)
    assert rc == 0 and rc2 == 0 and np.array_equal(xa, xc) and rel <= 1e-10
