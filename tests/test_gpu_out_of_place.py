"""The out-of-place form of the source update (mgrhd_options.E_g_out ...
v_out): the same results, bit for bit, as the update in place, the inputs
left unchanged, and cells the update leaves untouched copied through."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2407_18304_amd import mgrhd
from paper_2407_18304_amd import workloads as W

import gpu_util as U

pytestmark = pytest.mark.gpu


def _same(a, b):
    ga, gia, goa, gsa = a
    gb, gib, gob, gsb = b
    for k in U.FIELDS:
        assert np.array_equal(ga[k], gb[k], equal_nan=True), k
    assert np.array_equal(gia, gib) and np.array_equal(goa, gob) and np.array_equal(gsa, gsb)
    assert np.array_equal(a.trace, b.trace)


def _with_invalid_cells(w, rng):
    """Some cells with inputs the update rejects (left untouched)."""
    bad = rng.choice(w.n, size=max(3, w.n // 50), replace=False)
    st = w.state
    st["rho"][bad[0::3]] = -1.0
    st["E_g"][0, bad[1::3]] = np.nan
    st["F_g"][2, w.ng - 1, bad[2::3]] = np.inf
    return bad


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_out_of_place_equals_in_place(mode):
    rng = np.random.default_rng(11 + mode)
    for name, cells in (("config0", np.arange(4096)), ("config1", rng.choice(2 ** 21, 3000)),
                        ("config2", rng.choice(2 ** 24, 1500))):
        w = getattr(W, name)(cells=cells)
        bad = _with_invalid_cells(w, rng)
        a = U.run_gpu(w, mode)
        b = U.run_gpu(w, mode, out_of_place=True)
        _same(a, b)
        assert (b[3][bad] & mgrhd.ST_INVALID).all()
        for k in U.FIELDS:     # untouched cells: the inputs, copied through
            np.testing.assert_array_equal(b[0][k][..., bad], w.state[k][..., bad])
        U.compare(w, b, U.run_oracle(w, mode), label=f"{name} out of place, mode {mode}")


def test_out_of_place_every_variant():
    """Lane splits with one and several cells per wave, ragged and full."""
    w = W.config1(cells=np.arange(2000))
    default = mgrhd.get_variant(w.ng)
    try:
        for lpc, gpl, wps in [(16, 1, 0), (8, 2, 0), (4, 4, 0), (64, 1, 0), (8, 4, 0)]:
            mgrhd.set_variant(w.ng, lpc, gpl, wps)
            _same(U.run_gpu(w, 1), U.run_gpu(w, 1, out_of_place=True))
    finally:
        mgrhd.set_variant(w.ng, 0, 0)


def test_out_of_place_bad_table_copies_inputs():
    w = W.config0(cells=np.arange(300))
    w.edges = w.edges[::-1].copy()          # descending: rejected on the device
    g, gi, go, gs = U.run_gpu(w, 1, out_of_place=True)
    assert (gs == mgrhd.ST_BAD_TABLE).all()
    for k in U.FIELDS:
        assert np.array_equal(g[k], w.state[k])


def test_out_of_place_argument_errors():
    w = W.config0(cells=np.arange(10))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = {k: t(w.state[k]) for k in ("E_g", "F_g", "rho", "e_gas", "v")}
    tab = U.device_tables(w)
    outs = [torch.empty_like(st[k]) for k in U.FIELDS]
    # all four outputs or none
    o = mgrhd.default_options()
    o.E_g_out = outs[0].data_ptr()
    op = mgrhd.OpacityParams(w.ng, 1, tab["chi_lo"].data_ptr(), tab["alpha"].data_ptr(), None,
                             None)
    rc = mgrhd.lib().mgrhd_source_update(*(st[k].data_ptr() for k in
                                           ("E_g", "F_g", "rho", "e_gas", "v")), w.n,
                                         tab["edges"].data_ptr(), C.byref(op), w.dt, w.c_hat,
                                         None, C.byref(o))
    assert rc == mgrhd.E_NULL


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_out_of_place_temperature_dependent_opacity(mode):
    """The temperature-dependent kernels (the pulse test's opacity) out of
    place: the same bits as in place, the inputs unchanged."""
    w = W.config5(cells=np.arange(2500))
    rng = np.random.default_rng(21 + mode)
    bad = _with_invalid_cells(w, rng)
    a = U.run_gpu(w, mode)
    b = U.run_gpu(w, mode, out_of_place=True)
    _same(a, b)
    for k in U.FIELDS:
        np.testing.assert_array_equal(b[0][k][..., bad], w.state[k][..., bad])


@pytest.mark.parametrize("separate", [("F_g", "e_gas", "v"), ("E_g", "e_gas"), ("v",)])
def test_partly_in_place(separate):
    """Some arrays updated in place (output = input), the others into
    separate outputs: the same bits as fully in place, the separate inputs
    unchanged, and the untouched cells (invalid inputs, a rejected table)
    copied through into every separate output."""
    rng = np.random.default_rng(31)
    for mode in (0, 1):
        w = W.config1(cells=rng.choice(2 ** 21, 2500))
        bad = _with_invalid_cells(w, rng)
        a = U.run_gpu(w, mode)
        b = U.run_gpu(w, mode, out_of_place=separate)
        _same(a, b)
        for k in U.FIELDS:
            np.testing.assert_array_equal(b[0][k][..., bad], w.state[k][..., bad])
    w = W.config0(cells=np.arange(300))
    w.edges = w.edges[::-1].copy()          # descending: rejected on the device
    g, gi, go, gs = U.run_gpu(w, 1, out_of_place=separate)
    assert (gs == mgrhd.ST_BAD_TABLE).all()
    for k in U.FIELDS:
        assert np.array_equal(g[k], w.state[k])


def _imex(w, *, noalloc, out_of_place):
    """One IMEX step (workspace or no-allocation form) of workload w; with
    out_of_place, into NaN-filled outputs, checking the inputs are unchanged."""
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()
    st = {k: t(w.state[k]) for k in ("E_g", "F_g", "rho", "e_gas", "v")}
    outs = {k: torch.full_like(st[k], float("nan")) for k in U.FIELDS} if out_of_place else None
    status = torch.full((w.n,), -1, dtype=torch.int32, device="cuda")
    iters = torch.zeros(w.n, dtype=torch.int32, device="cuda")
    tab = U.device_tables(w)
    work = None if noalloc else torch.empty(mgrhd.imex_workspace_bytes(w.n, w.ng) // 8,
                                            dtype=torch.float64, device="cuda")
    mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"], tab["edges"],
                        tab["chi_lo"], alpha_chi=tab["alpha"], kappa_scale=tab["kappa"],
                        mean_mode=1, polish=1, dt=w.dt, c_hat=w.c_hat, c=w.c, a_rad=w.a_rad,
                        status=status, iters=iters, imex_work=work, imex_noalloc=noalloc,
                        out=None if outs is None else tuple(outs[k] for k in U.FIELDS))
    torch.cuda.synchronize()
    res = {k: st[k].cpu().numpy() for k in U.FIELDS}
    if outs is not None:
        for k in U.FIELDS:
            assert np.array_equal(res[k], w.state[k], equal_nan=True), f"input {k} modified"
            res[k] = outs[k].cpu().numpy()
    return res, iters.cpu().numpy(), status.cpu().numpy()


@pytest.mark.parametrize("noalloc", [False, True])
def test_imex_step_out_of_place(noalloc):
    """The IMEX step from U^(n) into separate outputs: the same bits as the
    step in place, U^(n) unchanged, untouched cells copied through."""
    rng = np.random.default_rng(41)
    w = W.config1(cells=rng.choice(2 ** 21, 4000))
    bad = _with_invalid_cells(w, rng)
    a, ia, sa = _imex(w, noalloc=noalloc, out_of_place=False)
    b, ib, sb = _imex(w, noalloc=noalloc, out_of_place=True)
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib)
    assert (sb[bad] & mgrhd.ST_INVALID).all()
    for k in U.FIELDS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
        np.testing.assert_array_equal(b[k][..., bad], w.state[k][..., bad])
    assert (np.abs(b["E_g"] - w.state["E_g"]) > 0).any()        # the step did something
