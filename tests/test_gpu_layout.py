"""Solver rows of grids with 129 or more vertices per axis are stored with
padded z lines (the first interior vertex of every line on a 128-byte
boundary).  These tests take every path through such rows against the FP64
oracle on identical draws:
- each smoother, coefficient mode and precision on a 17^3..129^3 hierarchy;
- tile heights and ragged x chunks on the 129^3 grid;
- the residual restricted along x by the pre-smoothing pass against the full
  residual and restriction;
- independent solves of mixed sizes (129 padded, 65 and 33 dense) through the
  packed output of mlsgd_solve_sizes;
- the unpacked state and adjoint outputs of mlsgd_solve_state_adjoint.
Bars as elsewhere: 1e-9 relative L2 (FP64), 1e-8 (FP32 V-cycles)."""
import numpy as np
import pytest

from paper_2606_09291_amd import inputs

pytestmark = pytest.mark.gpu

GRID = [17, 33, 65, 129]
M = [4, 2, 2, 1]
KW = dict(theta=1.0, alpha=1e-3, sigma2=2.0)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_09291_amd as m
    m.lib()
    return m


def _u_yd():
    n = GRID[-1]
    yd = inputs.target_sin(n)
    return inputs.control_xyz(n) + 15.0 * yd, yd


@pytest.fixture(scope="module")
def oracle_grad(orc):
    u, yd = _u_yd()
    pb = orc.make_problem(GRID, rtol=1e-13, **KW)
    go, so = orc.mlmc_gradient(pb, None, u, yd, M, first=[1, 1, 1, 1])
    return go, so


def _ctx(mm, precision="fp64", **extra):
    prec = {"fp64": mm.FP64, "mixed": mm.MIXED_FP32, "bf16": mm.MIXED_BF16}[precision]
    _, yd = _u_yd()
    return mm.Context(mm.Problem(grid_n=GRID, y_d=yd, rtol=1e-12, precision=prec, **KW, **extra),
                      use_tuned=False)


@pytest.mark.parametrize("env,precision", [
    ({}, "fp64"),                                                    # Chebyshev, fused first pass
    ({"MLSGD_SMOOTHER": "rbgs"}, "fp64"),                            # in-place red-black GS
    ({"MLSGD_SMOOTHER": "rbfused"}, "fp64"),                         # fused red-black sweeps
    ({"MLSGD_SMOOTHER": "cheb", "MLSGD_CACHE64": "0"}, "fp64"),      # coefficient regenerated
    ({}, "mixed"),
    ({"MLSGD_SMOOTHER": "rbfused"}, "mixed"),
    ({}, "bf16"),
])
def test_padded_hierarchy_matches_oracle(mm, oracle_grad, monkeypatch, env, precision):
    print("padded hierarchy", env, precision, flush=True)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    u, _ = _u_yd()
    ctx = _ctx(mm, precision)
    g, st = ctx.mlmc_gradient(u, M, first=[1, 1, 1, 1])
    ctx.close()
    go, so = oracle_grad
    assert st["nonconverged"] == 0
    assert _rel(g.cpu().numpy(), go) <= (1e-9 if precision == "fp64" else 1e-8)
    assert st["J"] == pytest.approx(so["J"], rel=1e-10)


@pytest.mark.parametrize("tuning", [{"tile_y": 4, "xchunk": 40}, {"tile_y": 16, "xchunk": 48},
                                    {"tile_y": 8, "xchunk": 128}])
def test_padded_tiles_match_oracle(mm, oracle_grad, tuning):
    print("padded tiles", tuning, flush=True)
    u, _ = _u_yd()
    ctx = _ctx(mm)
    ctx.set_tuning(**tuning)
    g, st = ctx.mlmc_gradient(u, M, first=[1, 1, 1, 1])
    ctx.close()
    assert st["nonconverged"] == 0
    assert _rel(g.cpu().numpy(), oracle_grad[0]) <= 1e-9


def _oracle_solve(orc, n, sample, level, f_value, K=4, sigma2=1.0):
    c = orc.kl_coeffs(0, level, sample, K, sigma2)
    b = inputs.constant(n, f_value)
    b[0] = b[-1] = 0
    b[:, 0] = b[:, -1] = 0
    b[:, :, 0] = b[:, :, -1] = 0
    # the FP64 residual floor of a 129^3 solve sits just above 1e-13
    x, _, rr = orc.solve(n, c, b, method=orc.SOLVE_MGPCG, rtol=2e-13)
    assert rr <= 2e-13
    return x


def test_padded_solve_sizes(mm, orc):
    sizes = [129, 33, 65, 129]
    print("solve_sizes", sizes, flush=True)
    ctx = mm.Context(mm.Problem(grid_n=[9, 17, 33, 65], y_d=inputs.target_sin(65), rtol=1e-12),
                     use_tuned=False)
    ys, st = ctx.solve_sizes(sizes, level=6, first=2, f_value=1.0)
    ctx.close()
    assert st["nonconverged"] == 0
    for j, n in enumerate(sizes):
        y = ys[j].cpu().numpy()
        assert y[0].max() == 0 and y[:, :, -1].max() == 0
        assert _rel(y, _oracle_solve(orc, n, 2 + j, 6, 1.0)) <= 1e-10


def test_padded_state_adjoint_outputs(mm, orc):
    print("state/adjoint 129", flush=True)
    u, yd = _u_yd()
    ctx = _ctx(mm)
    y, p, phi, st = ctx.solve_state_adjoint(3, 0, 5, 2, u)
    ctx.close()
    n = GRID[-1]
    for k in range(2):
        c = orc.kl_coeffs(0, 3, 5 + k, 4, KW["sigma2"])
        b = u.copy()
        b[0] = b[-1] = 0
        b[:, 0] = b[:, -1] = 0
        b[:, :, 0] = b[:, :, -1] = 0
        yo, _, _ = orc.solve(n, c, b, method=orc.SOLVE_MGPCG, rtol=1e-13)
        assert _rel(y[k].cpu().numpy(), yo) <= 1e-10
        r = yo - yd
        r[0] = r[-1] = 0
        r[:, 0] = r[:, -1] = 0
        r[:, :, 0] = r[:, :, -1] = 0
        po, _, _ = orc.solve(n, c, r, method=orc.SOLVE_MGPCG, rtol=1e-13)
        assert _rel(p[k].cpu().numpy(), po) <= 1e-10
        assert float(phi[k]) == pytest.approx(orc.misfit(n, yo, yd), rel=1e-9)


@pytest.mark.parametrize("grid,M,precision,tuning", [
    ([9, 17, 33], [16, 8, 4], "fp64", {}),
    ([9, 17, 33], [16, 8, 4], "mixed", {}),
    ([17, 33, 65], [8, 4, 3], "fp64", {}),
    ([17, 33, 65], [8, 4, 3], "mixed", {}),
    ([17, 33, 65], [8, 4, 3], "bf16", {}),
    (GRID, M, "fp64", {}),
    (GRID, M, "fp64", {"tile_y": 16, "xchunk": 40}),
    (GRID, M, "mixed", {"tile_y": 8, "xchunk": 24}),
])
def test_fused_passes_equal_level_by_level_passes(mm, orc, monkeypatch, grid, M, precision, tuning):
    """The one-pass pre-smoothing with its residual, the one-pass
    post-smoothing, and the one-kernel cycle from 9^3 down compute what the
    level-by-level passes compute (two-step pass and residual pass; step with
    the folded coarse-grid correction and plain step; every step, transfer
    and coarse solve below 17^3), with the same faces, neighbours and
    summation order; only the compiler's fused multiply-adds and the
    association of the trilinear prolongation may differ.  Whole estimates then agree to rounding (a wrong
    neighbour or plane would change the preconditioner and move the Krylov
    iterates, and the result, by about the solver tolerance) with identical
    iteration counts, and both match the oracle."""
    print("fused smoothing", grid, precision, tuning, flush=True)
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    u = inputs.control_xyz(nL) + 15.0 * yd
    prec = {"fp64": mm.FP64, "mixed": mm.MIXED_FP32, "bf16": mm.MIXED_BF16}[precision]
    out = []
    for flag in ("0", "1"):
        monkeypatch.setenv("MLSGD_PRE2R", flag)
        monkeypatch.setenv("MLSGD_POST2", flag)
        monkeypatch.setenv("MLSGD_VSMALL", flag)
        ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, rtol=1e-12, precision=prec, **KW),
                         use_tuned=False)
        if tuning:
            ctx.set_tuning(**tuning)
        g, st = ctx.mlmc_gradient(u, M, first=[2] * len(M))
        ctx.close()
        assert st["nonconverged"] == 0
        out.append((g.cpu().numpy(), st))
    d = _rel(out[1][0], out[0][0])
    print("fused vs separate: relative L2", d, "iterations", out[0][1]["iters_state"],
          out[1][1]["iters_state"], out[0][1]["iters_adjoint"], out[1][1]["iters_adjoint"],
          flush=True)
    assert d <= 1e-13
    assert out[0][1]["J"] == pytest.approx(out[1][1]["J"], rel=1e-14)
    assert out[0][1]["iters_state"] == out[1][1]["iters_state"]
    assert out[0][1]["iters_adjoint"] == out[1][1]["iters_adjoint"]
    if grid != GRID:
        pb = orc.make_problem(grid, rtol=1e-13, **KW)
        go, _ = orc.mlmc_gradient(pb, None, u, yd, M, first=[2] * len(M))
        assert _rel(out[1][0], go) <= (1e-9 if precision == "fp64" else 1e-8)


@pytest.mark.parametrize("grid,M,precision,tuning", [
    (GRID, M, "fp64", {}),
    (GRID, M, "mixed", {"tile_y": 16, "xchunk": 40}),
    ([17, 33, 65], [8, 4, 3], "bf16", {}),
    (GRID, M, "fp64", {"xchunk": 9}),
])
def test_half_restriction_equals_full_restriction(mm, orc, monkeypatch, grid, M, precision,
                                                  tuning):
    """The fused pre-smoothing pass may write its residual already restricted
    along x (every second plane), the restriction then finishing y and z.
    Full weighting is a product of one-dimensional weights, so both orders
    give the coarse right-hand side up to rounding: whole estimates agree to
    rounding with identical iteration counts, and match the oracle.  Chunks
    of odd length (9 planes: more than one chunk on every grid from 17^3 up)
    cannot split the coarse planes between chunks, keep the full residual
    and give identical bits."""
    print("half restriction", grid, precision, tuning, flush=True)
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    u = inputs.control_xyz(nL) + 15.0 * yd
    prec = {"fp64": mm.FP64, "mixed": mm.MIXED_FP32, "bf16": mm.MIXED_BF16}[precision]
    out = []
    for flag in ("0", "1"):
        monkeypatch.setenv("MLSGD_PRE2R_HALF", flag)
        ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, rtol=1e-12, precision=prec, **KW),
                         use_tuned=False)
        if tuning:
            ctx.set_tuning(**tuning)
        g, st = ctx.mlmc_gradient(u, M, first=[1] * len(M))
        ctx.close()
        assert st["nonconverged"] == 0
        out.append((g.cpu().numpy(), st))
    d = _rel(out[1][0], out[0][0])
    print("half vs full restriction: relative L2", d, "iterations", out[0][1]["iters_state"],
          out[1][1]["iters_state"], out[0][1]["iters_adjoint"], out[1][1]["iters_adjoint"],
          flush=True)
    if tuning.get("xchunk", 0) % 2 == 1:
        assert np.array_equal(out[0][0], out[1][0])
    assert d <= 1e-13
    assert out[0][1]["J"] == pytest.approx(out[1][1]["J"], rel=1e-14)
    assert out[0][1]["iters_state"] == out[1][1]["iters_state"]
    assert out[0][1]["iters_adjoint"] == out[1][1]["iters_adjoint"]
    if grid != GRID:
        pb = orc.make_problem(grid, rtol=1e-13, **KW)
        go, _ = orc.mlmc_gradient(pb, None, u, yd, M, first=[1] * len(M))
        assert _rel(out[1][0], go) <= 1e-8


def test_largest_grids(mm, orc):
    """The largest grids mlsgd_solve_sizes takes, solved to rtol 1e-10 (an
    FP64 solve cannot reach 1e-12 there: its attainable relative residual
    grows with the condition number of A, about h^-2, and is printed).
    513^3 (pitch 528): the oracle applies its own operator, built from its own
    vertex coefficients, to the unpacked solution, and the residual f - A y is
    at most 2e-10 of f.  1025^3 (pitch 1040, about 110 GB of solver rows): the
    solve converges and the library's FP64 true residual is within rtol."""
    import torch
    print("largest grids", flush=True)
    for rtol in (1e-12, 1e-10):
        ctx = mm.Context(mm.Problem(grid_n=[9, 17, 33, 65], y_d=inputs.target_sin(65), rtol=rtol),
                         use_tuned=False)
        ys, st = ctx.solve_sizes([513], level=6, first=4, f_value=1.0, allow_noconv=rtol < 1e-10)
        print("513^3 at rtol", rtol, st, flush=True)
        if rtol < 1e-10:
            ctx.close()
            continue
        assert st["nonconverged"] == 0
        y = ys[0].cpu().numpy()
        del ys
        n = 513
        assert y[0].max() == 0 and y[:, -1].max() == 0 and y[:, :, 0].max() == 0
        c = orc.kl_coeffs(0, 6, 4, 4, 1.0)
        r = (1.0 - orc.apply(n, c, y))[1:-1, 1:-1, 1:-1]
        rel = float(np.linalg.norm(r) / np.sqrt(r.size))
        print("513^3 oracle residual / |f|", rel, flush=True)
        assert rel <= 2e-10
        del y, r
        _, st = ctx.solve_sizes([1025], level=6, first=5, f_value=1.0, want_y=False)
        print("1025^3", st, flush=True)
        assert st["nonconverged"] == 0 and st["max_relres"] <= 1e-10
        ctx.close()
    torch.cuda.empty_cache()
