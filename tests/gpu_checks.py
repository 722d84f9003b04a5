"""Compare helpers shared by the GPU parity tests.

Compare rules (the target tolerances): dist equal everywhere; sigma bitwise
equal where the oracle's sigma < 2**53, else within 1e-12 relative (sums of
more than 2**53 are rounded, and the GPU adds parents in another order); BC
within 1e-9 relative (every dependency term is >= 0, so there is no
cancellation), with exact zeros where the oracle has zeros.
"""
import numpy as np

import oracle
import paper_2401_02472_amd as bcm

TWO53 = float(2 ** 53)


def check_bc(got, want, rtol=1e-9):
    want = np.asarray(want)
    assert got.shape == want.shape
    zero = want == 0
    assert np.all(got[zero] == 0), "BC must be exactly zero where the oracle's is"
    err = np.abs(got - want)
    bad = err > rtol * np.abs(want)
    assert not bad.any(), f"{bad.sum()} BC values off; worst rel " \
                          f"{(err[~zero] / np.abs(want[~zero])).max()}"


def check_sigma(got, want):
    exact = want < TWO53
    assert np.array_equal(got[exact], want[exact])
    big = ~exact
    if big.any():
        assert np.all(np.abs(got[big] - want[big]) <= 1e-12 * want[big])


def run_mode(G, sources, mode, **kw):
    """BC through bc_run_async with an explicit execution mode (host result)."""
    import torch
    out = torch.empty(G.n, dtype=torch.float64, device="cuda")
    G.run_async(np.asarray(sources, np.int32), out, bcm.make_options(mode, **kw))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def plain(G, sources, **kw):
    return run_mode(G, sources, bcm.BC_MODE_PLAIN, **kw)


def batched(G, sources, **kw):
    return run_mode(G, sources, bcm.BC_MODE_BATCHED, **kw)


def oracle_bc(g, sources):
    want, st = oracle.bc(g.row_ptr, g.col_idx, np.asarray(sources, np.int32))
    assert st == oracle.OK
    return want


def oracle_bc_ext(g, sources):
    """The extended-range (long double) oracle's BC."""
    want, st = oracle.bc_ext(g.row_ptr, g.col_idx, np.asarray(sources, np.int32))
    assert st == oracle.OK
    return want


def check_sigma_ext(got, sig_m, sig_e):
    """Exported sigma (double: infinite past double's range) against the
    extended oracle's sig_m * 2**sig_e: equal below 2**53, 1e-12 relative up to
    double's largest value, infinite beyond it."""
    with np.errstate(over="ignore"):
        want = np.ldexp(sig_m, sig_e)
    fits = np.isfinite(want)
    assert np.all(np.isposinf(got[~fits]))
    check_sigma(got[fits], want[fits])
