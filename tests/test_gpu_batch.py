"""The batched patch launch (mgrhd_batch_*): uneven AMR-like patches with their
own group counts, edges and tables in one persistent launch, direct and
replayed from a captured hipGraph.  Checked per patch against the single-table
entry point and against the oracle.  GPU only."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2407_18304_amd import mgrhd, synth
from paper_2407_18304_amd import workloads as W

import gpu_util as U

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _layouts(n=12):
    # small cubes so the oracle can check whole patches
    return W.patch_layouts(n_patches=n, sides=(4, 6, 8, 10), ngs=(8, 16, 32, 64))


def _patch_dicts(dps, with_out=True):
    out = []
    for dp in dps:
        n = dp.layout.n
        d = dict(dp.state)
        d.update(edges=dp.tables["edges"], chi_lo=dp.tables["chi_lo"], alpha_chi=dp.tables["alpha"],
                 kappa_scale=dp.kappa, dt=dp.dt, c_hat=dp.c_hat)
        if with_out:
            d.update(iters=torch.zeros(n, dtype=torch.int32, device="cuda"),
                     outer=torch.zeros(n, dtype=torch.int32, device="cuda"),
                     status=torch.full((n,), -1, dtype=torch.int32, device="cuda"),
                     trace=torch.full((20, n), -7, dtype=torch.int32, device="cuda"))
        out.append(d)
    return out


def _consts():
    u = W.UNITS["patches"]
    return dict(c=u["c"], a_rad=u["a_rad"])


# (groups per lane, item scope): items per wave, or per workgroup compiled for
# 3 or 2 waves per SIMD
TUNINGS = [(2, 0), (4, 0), (2, 1), (2, 2), (4, 2)]


@pytest.mark.parametrize("gpl,scope", TUNINGS)
def test_batch_matches_single_table_and_oracle(gpl, scope):
    layouts = _layouts()
    dps = synth.device_patches(layouts)
    inputs = [synth.patch_to_host(dp) for dp in dps]          # pristine inputs
    pd = _patch_dicts(dps)
    b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
    b.set_tuning(gpl, 0, 300)                                   # several items per patch
    b.set_item_scope(scope)
    assert b.get_item_scope() == scope
    assert b.n_cells == sum(L.n for L in layouts)
    b.run()
    torch.cuda.synchronize()
    for L, w, d in zip(layouts, inputs, pd):
        res = U.patch_result(d, 1)
        assert (res[3] >= 0).all()
        # the single-table entry point on the same patch (another lane split:
        # the group sums round in another order)
        U.compare(w, res, U.run_gpu(w, 1), label=f"patch {L.index} vs single table")
        # the oracle
        U.compare(w, res, U.run_oracle(w, 1), label=f"patch {L.index} vs oracle")


@pytest.mark.parametrize("scope", [0, 1])
def test_batch_graph_replay_matches_direct_run(scope):
    """Capture [counter clear -> persistent solver] once, replay it several
    times on restored inputs, with eager work between the replays: every
    replay equals the direct run bit for bit."""
    layouts = _layouts(8)
    dps = synth.device_patches(layouts)
    pristine = [{k: v.clone() for k, v in dp.state.items()} for dp in dps]
    pd = _patch_dicts(dps)
    b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
    b.set_tuning(4 if scope == 0 else 2, 0, 256)
    b.set_item_scope(scope)

    def restore():
        for dp, p in zip(dps, pristine):
            for k in ("E_g", "F_g", "e_gas", "v"):
                dp.state[k].copy_(p[k])

    b.run()
    torch.cuda.synchronize()
    ref = [{k: dp.state[k].clone() for k in ("E_g", "F_g", "e_gas", "v")} for dp in dps]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        restore()
        b.capture(stream.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        restore()
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        b.launch(stream.cuda_stream)
        stream.synchronize()
        for dp, r in zip(dps, ref):
            for k in r:
                assert torch.equal(dp.state[k], r[k]), (rep, k)
        del x


@pytest.mark.parametrize("scope", [0, 1])
def test_batch_ragged_and_empty_patches(scope):
    layouts = W.patch_layouts(n_patches=5, sides=(1, 3, 5), ngs=(1, 3, 8, 13, 33))
    dps = synth.device_patches(layouts)
    inputs = [synth.patch_to_host(dp) for dp in dps]
    pd = _patch_dicts(dps)
    # add an empty patch
    e = {k: v[..., :0].contiguous() for k, v in pd[0].items() if isinstance(v, torch.Tensor)
         and k not in ("edges", "chi_lo", "alpha_chi")}
    e.update(edges=pd[0]["edges"], chi_lo=pd[0]["chi_lo"], alpha_chi=pd[0]["alpha_chi"],
             dt=pd[0]["dt"], c_hat=pd[0]["c_hat"])
    b = mgrhd.Batch(pd + [e], mean_mode=2, polish=1, **_consts())
    b.set_item_scope(scope)
    b.run()
    torch.cuda.synchronize()
    for w, d in zip(inputs, pd):
        res = U.patch_result(d, 2)
        U.compare(w, res, U.run_oracle(w, 2), label=f"ragged patch N_g={w.ng} n={w.n}")


@pytest.mark.parametrize("gpl,scope", TUNINGS)
def test_batch_wide_patches(gpl, scope):
    """Patches wider than 64 groups (the kernels with 128-group table slots;
    at 2 groups per lane a cell spans the whole wavefront) next to narrow ones."""
    layouts = W.patch_layouts(n_patches=5, seed=78, sides=(2, 3), ngs=(8, 65, 100, 128))
    assert max(L.ng for L in layouts) > 64
    dps = synth.device_patches(layouts)
    inputs = [synth.patch_to_host(dp) for dp in dps]
    pd = _patch_dicts(dps)
    b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
    b.set_tuning(gpl, 0, 16)
    b.set_item_scope(scope)
    b.run()
    torch.cuda.synchronize()
    for w, d in zip(inputs, pd):
        res = U.patch_result(d, 1)
        assert (res[3] >= 0).all()
        U.compare(w, res, U.run_oracle(w, 1), label=f"wide patch N_g={w.ng} n={w.n}")


def test_batch_argument_errors():
    layouts = _layouts(2)
    dps = synth.device_patches(layouts)
    pd = _patch_dicts(dps)
    with pytest.raises(mgrhd.MgrhdError):
        mgrhd.Batch(pd, mean_mode=5)
    b = mgrhd.Batch(pd, mean_mode=1, **_consts())
    with pytest.raises(mgrhd.MgrhdError):
        b.set_tuning(3, 0, 100)
    for bad in (-1, 3):
        with pytest.raises(mgrhd.MgrhdError) as e:
            b.set_item_scope(bad)
        assert e.value.code == mgrhd.E_OPTION
    assert b.get_item_scope() == 1            # the default
    b.close()


@pytest.mark.parametrize("gpl,scope", TUNINGS)
def test_batch_bad_table_patch(gpl, scope):
    """A patch whose table is invalid (a negative group opacity) is flagged
    cell by cell and left unchanged; the patches around it are solved."""
    layouts = _layouts(6)
    dps = synth.device_patches(layouts)
    inputs = [synth.patch_to_host(dp) for dp in dps]
    pd = _patch_dicts(dps)
    bad = 2
    pd[bad]["chi_lo"] = pd[bad]["chi_lo"].clone()
    pd[bad]["chi_lo"][1] = -1.0
    b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
    b.set_tuning(gpl, 0, 100)
    b.set_item_scope(scope)
    b.run()
    torch.cuda.synchronize()
    for i, (w, d) in enumerate(zip(inputs, pd)):
        st = d["status"].cpu().numpy()
        if i == bad:
            assert (st == mgrhd.ST_BAD_TABLE).all()
            assert (d["iters"].cpu().numpy() == 0).all()
            for k in ("E_g", "F_g", "e_gas", "v"):
                assert np.array_equal(d[k].cpu().numpy(), w.state[k]), k
        else:
            assert (st >= 0).all() and (st != mgrhd.ST_BAD_TABLE).all()


def test_batch_warm_start_matches_plain():
    """One network per group count, trained on solver pairs of patches drawn
    with the training seed and attached to the batch; the warm-started batch
    (temperature guess, one fused inference launch per group count over all
    of its patches, equal to the per-patch launches) gives the plain batch's
    results, eagerly and replayed from the batch's graph holding the
    inference launches and the batched solve.  (Networks this small, trained on other patches' tables, need not
    save Newton steps: the step counts are printed, and the benchmark measures
    the gain of fully trained networks.)"""
    from paper_2407_18304_amd import warmstart
    ngs = (8, 16)
    nets = {}
    for ng in ngs:
        tl = W.patch_layouts(n_patches=4, seed=W.TRAIN_SEED, sides=(16,), ngs=(ng,))
        tdps = synth.device_patches(tl, seed=W.TRAIN_SEED)
        X, Y, ok = warmstart.make_training_data_patches(tdps)
        nets[ng] = warmstart.train(X, Y, ok, epochs=6, batch=1024, holdout=2048)
        assert nets[ng].history[-1] < nets[ng].history[0]
        del tdps, X, Y, ok
    layouts = W.patch_layouts(n_patches=8, sides=(6, 8, 10), ngs=ngs)
    dps = synth.device_patches(layouts)
    inputs = [synth.patch_to_host(dp) for dp in dps]
    pd = _patch_dicts(dps)
    b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
    b.run()
    torch.cuda.synchronize()
    keys = ("E_g", "F_g", "e_gas", "v")
    plain = [({k: d[k].cpu().numpy() for k in keys}, d["iters"].cpu().numpy(),
              d["status"].cpu().numpy()) for d in pd]
    guesses = [torch.empty(dp.layout.n, dtype=torch.float64, device="cuda") for dp in dps]
    bw = mgrhd.Batch([dict(d, guess=g) for d, g in zip(pd, guesses)], mean_mode=1, polish=1,
                     guess_kind=1, **_consts())
    pws = warmstart.PatchWarmStart(nets)
    stream = torch.cuda.Stream()

    def check(label):
        it_p, it_w = [], []
        for w, d, (gp, ip, sp), gt in zip(inputs, pd, plain, guesses):
            guess = gt.cpu().numpy()
            res = U.patch_result(d, 1, guess=guess, guess_kind=1)
            gw, iw, _, sw = res
            # the warm-started patch against the oracle given the same guess
            U.compare(w, res, U.run_oracle(w, 1, guess=guess, guess_kind=1),
                      label=f"{label}: warm patch N_g={w.ng} n={w.n}")
            # and the same root as plain Newton from the old state
            ok = (sp == 0) & (sw == 0)
            assert ok.mean() > 0.95, label
            for k, e in U.field_errors(w, gw, gp, ok).items():
                assert e < U.TOL, (label, k, e)
            it_p.append(ip[ok])
            it_w.append(iw[ok])
        ip, iw = np.concatenate(it_p), np.concatenate(it_w)
        print(f"{label}: Newton steps per cell plain {ip.mean():.3f}, warm {iw.mean():.3f}")

    # the per-patch inference (one launch per patch) for comparison
    synth.fill_patches(dps)
    per_patch = [torch.empty_like(g) for g in guesses]
    with torch.cuda.stream(stream):
        pws.guesses(dps, per_patch)
    stream.synchronize()
    pws.attach(bw)                            # one inference launch per group count
    synth.fill_patches(dps)                   # the same inputs again
    with torch.cuda.stream(stream):
        bw.infer(stream.cuda_stream)
    stream.synchronize()
    for g, q in zip(guesses, per_patch):      # same tiles, same kernel code
        assert torch.equal(g, q)
    synth.fill_patches(dps)
    with torch.cuda.stream(stream):
        bw.run(stream.cuda_stream)            # inference and solve
    stream.synchronize()
    check("eager")
    with torch.cuda.stream(stream):
        bw.capture(stream.cuda_stream)        # both in one graph
    torch.cuda.synchronize()
    for rep in range(2):
        synth.fill_patches(dps)
        for g in guesses:
            g.fill_(-1.0)                     # the replay must write them again
        x = torch.randn(1000, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            bw.launch(stream.cuda_stream)
        stream.synchronize()
        check(f"graph replay {rep}")
        del x
    bw.close()


def test_batch_full_size_sampled():
    """The benchmark's 2000-patch workload at full size (1.44e8 cells, about
    155 GB of state), drawn on the device and solved in the benchmark's
    launch configuration (the library's default tuning, captured in a graph
    and launched); sampled cells of sampled patches against the oracle on the
    same inputs."""
    layouts = W.patch_layouts()
    assert len(layouts) == 2000
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(len(layouts), 24, replace=False))
    dps = synth.device_patches(layouts)
    try:
        samples = {}
        for p in pick:
            n = layouts[p].n
            idx = np.sort(rng.choice(n, min(32, n), replace=False))
            samples[p] = (idx, synth.patch_to_host(dps[p], idx))    # pristine inputs
        pd = _patch_dicts(dps)
        b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            b.capture(stream.cuda_stream)
        b.launch(stream.cuda_stream)
        stream.synchronize()
        res = {}
        for p, (idx, w) in samples.items():
            res[p] = U.patch_result(pd[p], 1, idx)
        assert all(bool((d["status"] >= 0).all()) for d in pd)
        b.close()
    finally:
        del dps
        pd = None
        torch.cuda.empty_cache()
    # the oracle on all sampled cells at once per patch
    for p, (idx, w) in samples.items():
        U.compare(w, res[p], U.run_oracle(w, 1),
                  label=f"full-size batch: patch {p} (N_g={w.ng}), {len(idx)} sampled cells")


def test_batch_library_autotuner_reads_only():
    """mgrhd_batch_tune times its candidates on copies of a sample of every
    patch: the patches' arrays are unchanged, the chosen tuning is one of the
    candidates, and a run with it matches the oracle."""
    layouts = W.patch_layouts(n_patches=10, seed=33, sides=(8, 12, 16), ngs=(8, 16, 64))
    dps = synth.device_patches(layouts)
    inputs = [synth.patch_to_host(dp) for dp in dps]
    pd = _patch_dicts(dps)
    before = [{k: d[k].clone() for k in ("E_g", "F_g", "e_gas", "v", "iters", "status")}
              for d in pd]
    b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
    b.tune()
    for d, ref in zip(pd, before):
        for k, v in ref.items():
            assert torch.equal(d[k], v), k
    g, blocks, chunk = b.get_tuning()
    assert (g, b.get_item_scope(), chunk) in {(2, 0, 1024), (4, 0, 1024), (2, 1, 256),
                                              (2, 1, 1024), (2, 2, 256), (4, 2, 1024)}
    b.run()
    torch.cuda.synchronize()
    for w, d in zip(inputs, pd):
        res = U.patch_result(d, 1)
        U.compare(w, res, U.run_oracle(w, 1), label=f"tuned batch, patch N_g={w.ng} n={w.n}")


def test_batch_random_combinations():
    """Seeded random batches (patch counts, sides 1 ... 12, group counts
    1 ... 128, mean modes, groups per lane, item scopes, cells per item down
    to 7), every patch against the oracle."""
    rng = np.random.default_rng(3)
    for case in range(15):
        npat = int(rng.integers(2, 9))
        sides = tuple(int(x) for x in rng.choice([1, 2, 3, 5, 7, 9, 12], 3))
        ngs = tuple(int(x) for x in rng.choice([1, 2, 5, 8, 13, 16, 31, 32, 64, 65, 100, 128], 3))
        mode = int(rng.integers(0, 3))
        g = int(rng.choice([2, 4]))
        scope = int(rng.integers(0, 3))
        chunk = int(rng.choice([7, 64, 256, 1000]))
        layouts = W.patch_layouts(n_patches=npat, seed=1000 + case, sides=sides, ngs=ngs)
        dps = synth.device_patches(layouts)
        inputs = [synth.patch_to_host(dp) for dp in dps]
        pd = _patch_dicts(dps)
        b = mgrhd.Batch(pd, mean_mode=mode, polish=1, **_consts())
        b.set_tuning(g, 0, chunk)
        b.set_item_scope(scope)
        b.run()
        torch.cuda.synchronize()
        for w, d in zip(inputs, pd):
            res = U.patch_result(d, mode)
            assert (res[3] >= 0).all()
            U.compare(w, res, U.run_oracle(w, mode),
                      label=f"random batch {case} ({g},{scope},{chunk}): patch N_g={w.ng} n={w.n}")
        b.close()


@pytest.mark.parametrize("gpl,scope", TUNINGS)
def test_batch_out_of_place(gpl, scope):
    """Patches with their own output arrays (mgrhd_patch.E_g_out ... v_out),
    beside patches updated in place: the same bits as the whole batch in
    place, the inputs of the out-of-place patches unchanged, and a patch
    with a rejected table and cells with invalid inputs copied through."""
    layouts = _layouts(8)
    dps = synth.device_patches(layouts)
    bad_table, bad_cells = 2, 5
    runs = []
    for oop in (False, True):
        synth.fill_patches(dps)                                  # the same inputs twice
        pd = _patch_dicts(dps)
        pd[bad_table]["chi_lo"] = pd[bad_table]["chi_lo"].clone()
        pd[bad_table]["chi_lo"][1] = -1.0
        pd[bad_cells]["rho"] = pd[bad_cells]["rho"].clone()
        pd[bad_cells]["rho"][::7] = -1.0
        inputs = [{k: d[k].clone() for k in U.FIELDS} for d in pd]
        outs = []
        for i, d in enumerate(pd):
            if oop and i % 3 != 1:                               # every third stays in place
                o = {k: torch.full_like(d[k], float("nan")) for k in U.FIELDS}
                d["out"] = tuple(o[k] for k in U.FIELDS)
                outs.append(o)
            else:
                outs.append(None)
        b = mgrhd.Batch(pd, mean_mode=1, polish=1, **_consts())
        b.set_tuning(gpl, 0, 100)
        b.set_item_scope(scope)
        b.run()
        torch.cuda.synchronize()
        res = []
        for d, o, x in zip(pd, outs, inputs):
            if o is not None:
                for k in U.FIELDS:                               # inputs only read
                    assert torch.equal(d[k], x[k]), k
            src = o if o is not None else d
            res.append(({k: src[k].cpu().numpy() for k in U.FIELDS},
                        d["status"].cpu().numpy(), d["iters"].cpu().numpy()))
        runs.append((res, inputs))
        b.close()
    (a, _), (b_, inputs) = runs
    for i, ((ra, sa, ia), (rb, sb, ib)) in enumerate(zip(a, b_)):
        assert np.array_equal(sa, sb) and np.array_equal(ia, ib), i
        for k in U.FIELDS:
            assert np.array_equal(ra[k], rb[k]), (i, k)
    st = b_[bad_table][1]
    assert (st == mgrhd.ST_BAD_TABLE).all()
    for k in U.FIELDS:
        assert np.array_equal(b_[bad_table][0][k], inputs[bad_table][k].cpu().numpy()), k
    sc = b_[bad_cells][1]
    assert (sc[::7] & mgrhd.ST_INVALID).all()
    for k in U.FIELDS:
        assert np.array_equal(b_[bad_cells][0][k][..., ::7],
                              inputs[bad_cells][k].cpu().numpy()[..., ::7]), k


def test_batch_out_of_place_needs_all_four_outputs():
    dps = synth.device_patches(_layouts(2))
    pd = _patch_dicts(dps)
    o = torch.empty_like(pd[0]["E_g"])
    L = mgrhd._batch_lib()
    arr = (mgrhd.Patch * 1)()
    q = arr[0]
    d = pd[0]
    ng, n = d["E_g"].shape
    q.E_g, q.F_g, q.rho = d["E_g"].data_ptr(), d["F_g"].data_ptr(), d["rho"].data_ptr()
    q.e_gas, q.v = d["e_gas"].data_ptr(), d["v"].data_ptr()
    q.group_edges, q.chi_lo = d["edges"].data_ptr(), d["chi_lo"].data_ptr()
    q.alpha_chi = d["alpha_chi"].data_ptr()
    q.n_cells, q.n_groups, q.dt, q.c_hat = n, ng, float(d["dt"]), float(d["c_hat"])
    q.E_g_out = o.data_ptr()                                     # one of the four
    h = C.c_void_p()
    opt = mgrhd.default_options()
    assert L.mgrhd_batch_create(arr, 1, 1, C.byref(opt), C.byref(h)) == mgrhd.E_NULL
    assert not h.value
