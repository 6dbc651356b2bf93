"""mgrhd_imex_step_noalloc, the IMEX step for callers that cannot allocate:
through the C ABI it gives what mgrhd_imex_step with a caller workspace gives,
on two calls in a row (the second with fewer cells and groups), and device
memory stays as it was.  GPU only."""
import numpy as np
import pytest
import torch

from paper_2407_18304_amd import mgrhd
from paper_2407_18304_amd import workloads as W

import gpu_util as U

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _step(w, noalloc, work=None):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()
    st = {k: t(w.state[k]) for k in ("E_g", "F_g", "rho", "e_gas", "v")}
    status = torch.full((w.n,), -1, dtype=torch.int32, device="cuda")
    iters = torch.zeros(w.n, dtype=torch.int32, device="cuda")
    tab = U.device_tables(w)
    mgrhd.source_update(st["E_g"], st["F_g"], st["rho"], st["e_gas"], st["v"], tab["edges"],
                        tab["chi_lo"], alpha_chi=tab["alpha"], kappa_scale=tab["kappa"],
                        mean_mode=1, polish=1, dt=w.dt, c_hat=w.c_hat, c=w.c, a_rad=w.a_rad,
                        status=status, iters=iters, imex_work=work, imex_noalloc=noalloc)
    torch.cuda.synchronize()
    return ({k: v.cpu().numpy() for k, v in st.items()}, iters.cpu().numpy(),
            status.cpu().numpy())


def test_noalloc_imex_step_matches_workspace_step():
    cases = [W.config1(cells=np.arange(20000)),                  # 10.9 MB of U^(n+1/2)
             W.config2(cells=np.arange(3000), ng=24)]            # smaller, other group count
    for w in cases:
        need = mgrhd.imex_workspace_bytes(w.n, w.ng)
        work = torch.empty(need // 8, dtype=torch.float64, device="cuda")
        ref, it_r, st_r = _step(w, False, work)
        free0 = torch.cuda.mem_get_info()[0]
        got, it_g, st_g = _step(w, True)
        free1 = torch.cuda.mem_get_info()[0]
        assert (st_r >= 0).all() and np.array_equal(st_g, st_r)
        assert np.array_equal(it_g, it_r)
        # same kernels on the same inputs: identical results
        for k in U.FIELDS:
            assert np.array_equal(got[k], ref[k]), k
        assert (np.abs(got["E_g"] - w.state["E_g"]) > 0).any()       # the step did something
        # the call allocated nothing (torch's own tensors of _step are freed
        # to torch's cache, which keeps device memory reserved either way)
        assert free1 >= free0 - (64 << 20), (free0, free1)


def test_noalloc_imex_step_rejects_oversize_input():
    w = W.config1(cells=np.arange(130000))          # 71 MB of U^(n+1/2) > 32 MiB
    assert mgrhd.imex_workspace_bytes(w.n, w.ng) > 8 * 4 * 1024 * 1024
    with pytest.raises(mgrhd.MgrhdError) as e:
        _step(w, True)
    assert e.value.code == mgrhd.E_SIZE


def test_noalloc_imex_step_at_its_limit():
    """61 680 cells of 16 groups (4 N_g + 4 = 68 doubles each) fill the
    32 MiB array; one more cell is refused with nothing enqueued."""
    limit = 4 * 1024 * 1024 // 68
    w = W.config1(cells=np.arange(limit + 1))
    assert mgrhd.imex_workspace_bytes(w.n, w.ng) > 8 * 4 * 1024 * 1024
    with pytest.raises(mgrhd.MgrhdError) as e:
        _step(w, True)
    assert e.value.code == mgrhd.E_SIZE
    w = W.config1(cells=np.arange(limit))
    assert mgrhd.imex_workspace_bytes(w.n, w.ng) <= 8 * 4 * 1024 * 1024
    work = torch.empty(mgrhd.imex_workspace_bytes(w.n, w.ng) // 8, dtype=torch.float64,
                       device="cuda")
    ref, it_r, st_r = _step(w, False, work)
    got, it_g, st_g = _step(w, True)
    assert np.array_equal(st_g, st_r) and np.array_equal(it_g, it_r)
    for k in U.FIELDS:
        assert np.array_equal(got[k], ref[k]), k
