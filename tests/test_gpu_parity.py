"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances (FP32 populations vs FP64 oracle): relative L2 over fluid cells
<= 1e-5 per velocity channel; <= 1e-4 on quadrature mean and standard
deviation.  Every comparison uses the same seeded inputs on both sides.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2508_18202_amd import inputs
from paper_2508_18202_amd import lbmsc as L
from paper_2508_18202_amd import sc
from gpu_util import oracle_case, per_channel_maxrel, per_channel_rel, rel_l2

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5
MOMENT_TOL = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _ensemble(w, solid, thetas, probes=None, **kw):
    cg = sc.make_geometry(w, solid, probes)
    return sc.Ensemble([cg], [thetas], **kw), cg


@pytest.mark.parametrize("model", ["bgk", "smagorinsky", "rr3"])
def test_step_by_step_populations(model):
    """Every step of a small case with all boundary kinds: populations after
    1, 2, 3, 4 and 9 steps (both storage parities) against the oracle."""
    _say(f"step-by-step {model}")
    w = inputs.scaled(inputs.urban_les(), 24, 12, 10, model=model, tau0=0.56, cs=0.12 if model != "bgk" else 0.0,
                      ramp=5)
    solid = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    solid[0:5, 3:7, 7:11] = 1
    solid[0:3, 8:10, 14:16] = 1
    theta = (0.012, math.radians(4.0), 0.5)
    ens, cg = _ensemble(w, solid, [theta])
    case = oracle_case(w, solid, theta)
    f = case.init()
    _, wl, _ = orc.lattice()
    fluid = cg.fluid
    done = 0
    try:
        for target in (1, 2, 3, 4, 9):
            ens.advance(target - done)
            while done < target:
                f = case.step(done, f)
                done += 1
            g = ens.populations(0).cpu().numpy().astype(np.float64)
            ref = f - wl[:, None]
            # the raw slots of solid cells (swapped by even steps, filled by
            # odd steps) carry no state and stay at zero
            raw = ens.f[0].view(19, cg.qs)[:, : cg.ncells].cpu().numpy()
            assert not np.any(raw[:, ~fluid]), target
            err = np.abs(g[:, fluid] - ref[:, fluid]).max()
            scale = np.abs(ref[:, fluid]).max()
            assert err <= 1e-5 * scale + 1e-9, (target, err, scale)
            u = ens.fields(0).cpu().numpy()
            o = orc.qoi_fields(case, f)
            for k, e in enumerate(per_channel_rel(u, o, fluid)[:3]):
                assert e < FIELD_TOL, (target, k, e)
    finally:
        ens.close()


def test_small_block_full_parity():
    """Small case (BGK tau 0.6, 32x16x16, one block, 5 Gauss-Legendre nodes,
    1000 steps): final velocity fields per node and their moments."""
    w = inputs.small_block()
    solid = inputs.solid_mask(w)
    _say("small block: GPU")
    r = sc.run_sc(w, solid)
    ens = r["ensemble"]
    try:
        q = r["q"].cpu().numpy()
        fluid = r["geometry"].fluid
        x, a = orc.collocation(w)
        assert np.abs(r["weights"] - a).max() < 1e-14
        qo = []
        for j, xi in enumerate(x):
            _say(f"small block: oracle node {j}")
            th = orc.node_params(w, xi)
            res = orc.run(oracle_case(w, solid, th), w.steps)
            qo.append(res["final"])
            errs = per_channel_rel(q[j], res["final"], fluid)
            assert max(errs) < FIELD_TOL, (j, errs)
        qo = np.stack(qo)                       # [nodes, 4, cells]
        eo, vo = orc.moments(qo, a)
        mean = r["mean"].cpu().numpy().T        # [4, cells]
        var = r["var"].cpu().numpy().T
        for k in range(4):
            assert rel_l2(mean[k], eo[k], fluid) < MOMENT_TOL
            assert rel_l2(np.sqrt(np.maximum(var[k], 0)), np.sqrt(np.maximum(vo[k], 0)), fluid) < MOMENT_TOL
        assert r["n_negative"] == 0            # Gauss-Legendre weights are positive
    finally:
        ens.close()


@pytest.mark.parametrize("ramp", [1000, 40])
def test_urban_les_short_horizon(ramp):
    """Urban LES recipe (Smagorinsky Cs 0.1, log-law inflow, 13 Smolyak nodes)
    on a reduced 64x32x24 box, 200 steps, time averages over the last 50."""
    w = inputs.scaled(inputs.urban_les(steps=200, avg_len=50), 64, 32, 24, ramp=ramp)
    solid = inputs.solid_mask(w)
    _say(f"urban short ramp={ramp}: GPU")
    r = sc.run_sc(w, solid)
    ens = r["ensemble"]
    try:
        q = r["q"].cpu().numpy()
        fluid = r["geometry"].fluid
        x, a = orc.collocation(w)
        qo = []
        for j, xi in enumerate(x):
            th = orc.node_params(w, xi)
            res = orc.run(oracle_case(w, solid, th), w.steps, avg_start=w.avg_start)
            qo.append(res["avg"])
            errs = per_channel_rel(q[j], res["avg"], fluid)
            assert max(errs) < FIELD_TOL, (j, errs)
        qo = np.stack(qo)
        eo, vo = orc.moments(qo, a)
        mean = r["mean"].cpu().numpy().T
        var = r["var"].cpu().numpy().T
        for k in range(4):
            assert rel_l2(mean[k], eo[k], fluid) < MOMENT_TOL, k
            so = np.sqrt(np.maximum(vo[k], 0))
            assert rel_l2(np.sqrt(np.maximum(var[k], 0)), so, fluid) < MOMENT_TOL, k
    finally:
        ens.close()


def test_full_size_urban_first_steps():
    """The bench launch configuration (13 nodes of 256x128x64 in one plan,
    graph replay on): the first 24 steps of every node against the oracle at
    full size."""
    w = inputs.urban_les()
    solid = inputs.solid_mask(w)
    x, a, th = sc.collocation(w)
    cg = sc.make_geometry(w, solid)
    w0 = inputs.scaled(w, w.nx, w.ny, w.nz, ramp=0)   # full inflow from step 0
    cg.w = w0
    ens = sc.Ensemble([cg], [th], use_graph=True)
    try:
        _say("full-size urban: GPU 24 steps")
        ens.advance(24)
        fluid = cg.fluid
        xo, ao = orc.collocation(w)
        for j in range(len(th)):
            _say(f"full-size urban: oracle node {j}")
            tho = orc.node_params(w, xo[j])
            case = oracle_case(w0, solid, tho)
            res = orc.run(case, 24)
            u = ens.fields(j).cpu().numpy()
            errs = per_channel_rel(u, res["final"], fluid)
            mx = per_channel_maxrel(u, res["final"], fluid)
            _say(f"full-size urban node {j}: rel L2 {['%.2e' % e for e in errs]}, max {['%.2e' % e for e in mx]}")
            assert max(errs) < FIELD_TOL, (j, errs)
            assert max(mx) < 1e-4, (j, mx)
        assert ens.health() == -1
    finally:
        ens.close()


def test_moments_kernel_against_oracle():
    rng = np.random.default_rng(3)
    for nq in (1, 5, 13, 32, 40, 121):
        q = rng.standard_normal((nq, 1000, 4)).astype(np.float32) * 0.01 + 0.05
        if nq == 13:
            _, a = orc.smolyak_cc(2, 2)
        elif nq == 5:
            _, a = orc.gauss_legendre(5)
        else:
            a = rng.random(nq)
            a /= a.sum()
        qt = torch.from_numpy(q).cuda()
        mean, var, nneg = sc.moments(qt, a, count_negative=True)
        eo, vo = orc.moments(q.astype(np.float64), a)
        assert np.abs(mean.cpu().numpy() - eo).max() < 1e-15 * 100
        assert np.abs(var.cpu().numpy() - vo).max() < 1e-13 * max(1e-30, np.abs(vo).max()) + 1e-18
        assert nneg == int((vo < 0).sum())
    # empty input and bad weights
    mean, var = sc.moments(torch.zeros(3, 0, device="cuda"), np.array([0.2, 0.3, 0.5]))
    with pytest.raises(L.LbmError):
        sc.moments(torch.zeros(3, 10, device="cuda"), np.array([0.2, 0.3, 0.6]))


def test_moments_kernel_layouts():
    """The moments kernel's element paths against the oracle: groups of four
    (the vector path), a count not divisible by 4 (the per-element tail), a
    4-byte-offset buffer (per-element path only), and more elements than one
    pass of the grid covers (grid-stride)."""
    rng = np.random.default_rng(5)
    _, a13 = orc.smolyak_cc(2, 2)
    s = sc.stream_handle()
    for nq, n, offset in ((13, 3003, 0), (5, 4001, 0), (13, 4000, 1), (40, 2002, 1), (13, 4 * 4096 * 256 + 12, 0)):
        a = a13 if nq == 13 else rng.random(nq)
        a = a / a.sum()
        q = (rng.standard_normal((nq, n)) * 0.01 + 0.05).astype(np.float32)
        buf = torch.zeros(nq * n + offset, dtype=torch.float32, device="cuda")
        buf[offset:] = torch.from_numpy(q.reshape(-1)).cuda()
        mean = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        var = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        neg = torch.zeros(1, dtype=torch.int64, device="cuda")
        L.lbm_sc_moments(buf.data_ptr() + 4 * offset, np.ascontiguousarray(a, dtype=np.float64), nq, n,
                         mean.data_ptr() + 8 * offset, var.data_ptr() + 8 * offset, neg.data_ptr(), s)
        eo, vo = orc.moments(q.astype(np.float64), a)
        m = mean.cpu().numpy()[offset:offset + n]
        v = var.cpu().numpy()[offset:offset + n]
        assert np.abs(m - eo).max() < 1e-13, (nq, n, offset)
        assert np.abs(v - vo).max() < 1e-13 * np.abs(vo).max() + 1e-18, (nq, n, offset)
        assert int(neg.item()) == int((vo < 0).sum()), (nq, n, offset)


@pytest.mark.parametrize("inflow", ["loglaw", "series"])
def test_cache_blocks_equal_the_batched_order(inflow):
    """Steps advanced one instance block at a time (plain stretches from
    graphs, ramp, blend and window steps in chunks) give bitwise the
    populations and window averages of the whole batch per step (three
    blocks of five nodes; a window of 150 states, flushed every 64)."""
    if inflow == "loglaw":
        w = inputs.scaled(inputs.urban_les(steps=220, avg_len=150), 48, 24, 20, ramp=10)
    else:
        w = inputs.scaled(inputs.urban_series(hours=3, hour_steps=40, blend_steps=15), 48, 24, 20, ramp=10,
                          steps=220, avg_start=70)
    solid = inputs.solid_mask(w)
    probes = inputs.probe_cells(w, solid)
    cg = sc.make_geometry(w, solid, probes)
    x, a, th = sc.collocation(w)
    per_inst = 19 * 4 * cg.qs + 5 * cg.ncells
    out = {}
    for budget in (0, 2 * per_inst + 1):
        ens = sc.Ensemble([cg], [th[:5]], avg_begin=w.avg_start, avg_end=w.steps, use_graph=True,
                          variant=(128, 1, 1, 1), cache_block=budget)
        try:
            assert L.lbm_plan_cache_blocks(ens.plan) == (0 if budget == 0 else 3)
            ens.advance(w.steps)
            assert ens.health() == -1
            res = []
            for i in range(len(ens)):
                q = torch.empty(cg.ncells, 4, dtype=torch.float32, device="cuda")
                pq = torch.empty(len(probes), dtype=torch.float32, device="cuda")
                ens.averages_into(i, q, pq)
                res.append((ens.populations(i).cpu().numpy(), q.cpu().numpy(), pq.cpu().numpy()))
            out[budget] = res
        finally:
            ens.close()
    (r0, r1) = out.values()
    for i in range(5):
        for u, v in zip(r0[i], r1[i]):
            assert np.array_equal(u, v), i
    assert np.abs(r0[0][1]).max() > 0
    ens = sc.Ensemble([cg], [th[:2]], use_graph=True)
    try:
        with pytest.raises(L.LbmError):
            L.lbm_plan_set_cache_block(ens.plan, -1)
    finally:
        ens.close()


def test_batched_uneven_matches_one_at_a_time():
    """Three box sizes x three nodes in one plan equal the same instances run
    as separate plans, bit for bit, and each matches the oracle."""
    sizes = [(32, 16, 12), (48, 24, 16), (64, 32, 20)]
    base = inputs.uneven_cases(steps=60)[0]
    cases, thetas, ws, solids = [], [], [], []
    xo, ao = orc.collocation(base)
    sel = [0, 6, 12]
    for k, (nx, ny, nz) in enumerate(sizes):
        wk = inputs.scaled(base, nx, ny, nz, ramp=10)
        sk = inputs.building_array_mask(nx, ny, nz, 3, 2, 77 + k)
        ws.append(wk)
        solids.append(sk)
        cases.append(sc.make_geometry(wk, sk))
        thetas.append([orc.node_params(wk, xo[j]) for j in sel])
    ens = sc.Ensemble(cases, thetas, use_graph=False)
    try:
        ens.advance(60)
        batched = [ens.populations(i).cpu().numpy().copy() for i in range(len(ens))]
    finally:
        ens.close()
    i = 0
    for k in range(3):
        for j in range(3):
            single = sc.Ensemble([sc.make_geometry(ws[k], solids[k])], [[thetas[k][j]]], use_graph=False)
            try:
                single.advance(60)
                s = single.populations(0).cpu().numpy()
                assert np.array_equal(s, batched[i]), (k, j)
                if j == 1:
                    res = orc.run(oracle_case(ws[k], solids[k], thetas[k][j]), 60)
                    u = single.fields(0).cpu().numpy()
                    errs = per_channel_rel(u, res["final"], solids[k].reshape(-1) == 0)
                    assert max(errs) < FIELD_TOL, (k, errs)
            finally:
                single.close()
            i += 1


@pytest.mark.parametrize("cache_block", [None, 4 << 20])
def test_autotune_restores_state(tmp_path, monkeypatch, cache_block):
    """The launch-shape autotuner times every shape on the live batch (with
    4 MiB instance blocks: one instance per block, each block through its own
    step pairs) and then restores populations and step counter: continuing
    afterwards gives the same populations bit for bit as a plan that was
    never tuned; the second call is served from the cache file, written into
    directories the library creates."""
    cache = tmp_path / "cache" / "lbmsc" / "tune.json"
    monkeypatch.setenv("LBMSC_TUNE_CACHE", str(cache))
    w = inputs.scaled(inputs.urban_les(), 64, 32, 24, ramp=4)
    solid = inputs.solid_mask(w)
    _, _, th = sc.collocation(w)
    outs = []
    for tune in (False, True):
        ens, _ = _ensemble(w, solid, th[:3], variant=(256, 1, 0, 0), use_graph=tune, cache_block=cache_block)
        try:
            assert L.lbm_plan_cache_blocks(ens.plan) == (0 if cache_block is None else 3)
            ens.advance(6)
            before = [ens.populations(i).cpu().numpy() for i in range(3)]
            if tune:
                v = L.lbm_plan_autotune(ens.plan, sc.stream_handle())
                assert v[0] in (64, 128, 256, 512) and v[1] in (1, 2, 4) and 0 <= v[2] <= 3 and v[3] in (0, 1)
                assert L.lbm_plan_variant(ens.plan) == v
                assert L.lbm_plan_step(ens.plan) == 6
                for a, b in zip(before, [ens.populations(i).cpu().numpy() for i in range(3)]):
                    assert np.array_equal(a, b)
                assert L.lbm_plan_autotune(ens.plan, sc.stream_handle()) == v     # cached
                assert cache.exists() and '"' in cache.read_text()
            ens.advance(31)
            assert ens.health() < 0
            outs.append([ens.populations(i).cpu().numpy() for i in range(3)])
        finally:
            ens.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", [(128, 1, 0, 0), (512, 1, 1, 1), (128, 2, 2, 0), (256, 2, 3, 1), (512, 2, 0, 0),
                                     (64, 1, 1, 0), (64, 4, 2, 0), (128, 4, 3, 1), (512, 4, 1, 0)])
def test_launch_shapes_and_graphs_bitwise(variant):
    """Every launch shape (threads per workgroup, cells per thread,
    non-temporal) and graph replay give the same populations bit for bit."""
    w = inputs.scaled(inputs.urban_les(), 64, 32, 24, ramp=4)
    solid = inputs.solid_mask(w)
    _, _, th = sc.collocation(w)
    outs = []
    for kw in (dict(variant=(256, 1, 0, 0), use_graph=False), dict(variant=variant, use_graph=True)):
        ens, _ = _ensemble(w, solid, th[:3], **kw)
        try:
            ens.advance(57)
            outs.append([ens.populations(i).cpu().numpy() for i in range(3)])
        finally:
            ens.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_unstable_instance_is_isolated():
    """A node whose populations are poisoned is reported by the health check;
    the other nodes of the batch are bit-identical to a batch without it."""
    w = inputs.scaled(inputs.urban_les(), 32, 16, 12, ramp=0)
    solid = inputs.solid_mask(w)
    _, _, th = sc.collocation(w)
    ens, cg = _ensemble(w, solid, th[:3], use_graph=False)
    ref, _ = _ensemble(w, solid, th[:3], use_graph=False)
    try:
        c = int(np.flatnonzero(cg.fluid)[len(np.flatnonzero(cg.fluid)) // 2])   # a fluid cell
        ens.f[1][5 * cg.qs + c] = float("nan")
        ens.advance(10)
        ref.advance(10)
        assert ens.health() == 1
        assert ref.health() == -1
        for i in (0, 2):
            assert np.array_equal(ens.populations(i).cpu().numpy(), ref.populations(i).cpu().numpy())
    finally:
        ens.close()
        ref.close()


def test_series_inflow_step_by_step():
    """Time-dependent inflow from an hourly series (short hours: ramp 2, three
    steps per hour, two blending steps): populations after every hour change
    and into the held tail, against the oracle."""
    _say("series inflow step-by-step")
    w = inputs.scaled(inputs.urban_series(hours=4, hour_steps=3, blend_steps=2), 24, 12, 10, ramp=2,
                      tau0=0.56, ref_height=10.0)
    solid = np.zeros((w.nz, w.ny, w.nx), np.uint8)
    solid[0:5, 3:7, 7:11] = 1
    theta = (1.06, math.radians(3.0), 0.1)
    ens, cg = _ensemble(w, solid, [theta])
    case = oracle_case(w, solid, theta)
    f = case.init()
    _, wl, _ = orc.lattice()
    fluid = cg.fluid
    done = 0
    try:
        for target in (1, 3, 5, 6, 7, 9, 12, 17):
            ens.advance(target - done)
            while done < target:
                f = case.step(done, f)
                done += 1
            g = ens.populations(0).cpu().numpy().astype(np.float64)
            ref = f - wl[:, None]
            err = np.abs(g[:, fluid] - ref[:, fluid]).max()
            assert err <= 1e-5 * np.abs(ref[:, fluid]).max() + 1e-9, (target, err)
    finally:
        ens.close()


def test_series_graph_replay_matches_launches():
    """Graph replay starts only once the series inflow is constant: through
    the hours and into the held tail, graphs and plain launches agree bit for
    bit."""
    w = inputs.scaled(inputs.urban_series(hours=3, hour_steps=24, blend_steps=10), 64, 32, 24, ramp=12,
                      ref_height=24.0)
    solid = inputs.solid_mask(w)
    _, _, th = sc.collocation(w)
    outs = []
    for graph in (False, True):
        ens, _ = _ensemble(w, solid, th[:2], variant=(128, 2, 1, 0), use_graph=graph)
        try:
            got = []
            for n in (40, 96, 140):
                ens.advance(n - L.lbm_plan_step(ens.plan))
                got.append([ens.populations(i).cpu().numpy() for i in range(2)])
            outs.append(got)
        finally:
            ens.close()
    for a, b in zip(*outs):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_series_urban_short_horizon():
    """The urban recipe driven by an hourly series (13 Smolyak nodes on the
    speed multiplier and direction offset), 200 steps with an hour every 40
    steps, averages over the last 50: fields and moments against the oracle."""
    w = inputs.scaled(inputs.urban_series(hours=6, hour_steps=40, blend_steps=15), 64, 32, 24, ramp=20,
                      steps=200, avg_start=150, ref_height=24.0)
    solid = inputs.solid_mask(w)
    _say("series urban short: GPU")
    r = sc.run_sc(w, solid)
    ens = r["ensemble"]
    try:
        q = r["q"].cpu().numpy()
        fluid = r["geometry"].fluid
        x, a = orc.collocation(w)
        qo = []
        for j, xi in enumerate(x):
            th = orc.node_params(w, xi)
            res = orc.run(oracle_case(w, solid, th), w.steps, avg_start=w.avg_start)
            qo.append(res["avg"])
            errs = per_channel_rel(q[j], res["avg"], fluid)
            assert max(errs) < FIELD_TOL, (j, errs)
        eo, vo = orc.moments(np.stack(qo), a)
        mean = r["mean"].cpu().numpy().T
        var = r["var"].cpu().numpy().T
        for k in range(4):
            assert rel_l2(mean[k], eo[k], fluid) < MOMENT_TOL
            assert rel_l2(np.sqrt(np.maximum(var[k], 0)), np.sqrt(np.maximum(vo[k], 0)), fluid) < MOMENT_TOL
    finally:
        ens.close()


def test_rr3_urban_short_horizon():
    """The regularised third-order collision with the Smagorinsky tau_eff on
    the urban recipe (64x32x24, 13 Smolyak nodes, log-law inflow), 200 steps,
    time averages over the last 50, against the oracle: fields and moments."""
    w = inputs.scaled(inputs.urban_les(steps=200, avg_len=50), 64, 32, 24, ramp=40, model="rr3")
    solid = inputs.solid_mask(w)
    _say("rr3 urban short: GPU")
    r = sc.run_sc(w, solid)
    ens = r["ensemble"]
    try:
        q = r["q"].cpu().numpy()
        fluid = r["geometry"].fluid
        x, a = orc.collocation(w)
        qo = []
        for j, xi in enumerate(x):
            th = orc.node_params(w, xi)
            res = orc.run(oracle_case(w, solid, th), w.steps, avg_start=w.avg_start)
            qo.append(res["avg"])
            errs = per_channel_rel(q[j], res["avg"], fluid)
            assert max(errs) < FIELD_TOL, (j, errs)
        eo, vo = orc.moments(np.stack(qo), a)
        mean = r["mean"].cpu().numpy().T
        var = r["var"].cpu().numpy().T
        for k in range(4):
            assert rel_l2(mean[k], eo[k], fluid) < MOMENT_TOL
            assert rel_l2(np.sqrt(np.maximum(var[k], 0)), np.sqrt(np.maximum(vo[k], 0)), fluid) < MOMENT_TOL
    finally:
        ens.close()


@pytest.mark.parametrize("variant", [(128, 2, 1, 0), (64, 4, 3, 1), (512, 1, 2, 0)])
def test_rr3_launch_shapes_bitwise(variant):
    """The regularised collision gives the same populations bit for bit in
    every launch shape and under graph replay."""
    w = inputs.scaled(inputs.urban_les(), 64, 32, 24, ramp=4, model="rr3")
    solid = inputs.solid_mask(w)
    _, _, th = sc.collocation(w)
    outs = []
    for kw in (dict(variant=(256, 1, 0, 0), use_graph=False), dict(variant=variant, use_graph=True)):
        ens, _ = _ensemble(w, solid, th[:2], **kw)
        try:
            ens.advance(33)
            outs.append([ens.populations(i).cpu().numpy() for i in range(2)])
        finally:
            ens.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_rejections():
    w = inputs.small_block()
    solid = inputs.solid_mask(w).copy()
    solid[:, :, w.nx - 1] = 1                     # solid in the outflow column
    cg = sc.make_geometry(w, solid)
    f = torch.empty(19 * cg.qs, device="cuda")
    with pytest.raises(L.LbmError):
        sc.init_populations(cg, f)
    good = sc.make_geometry(inputs.scaled(w, w.nx, w.ny, w.nz, tau0=0.5), inputs.solid_mask(w))
    with pytest.raises(L.LbmError):               # tau0 <= 1/2
        sc.Ensemble([good], [[(0.05, 0.0, 0.0)]])
    ok = sc.make_geometry(w, inputs.solid_mask(w))
    for v in ((96, 1, 0, 0), (1024, 1, 0, 0), (128, 3, 0, 0), (128, 1, 4, 0), (128, 1, 0, 2), (128, 1, 0, -1)):
        with pytest.raises(L.LbmError):           # launch shapes outside the compiled set
            sc.Ensemble([ok], [[(0.05, 0.0, 0.0)]], variant=v)


@pytest.mark.parametrize("nx,ny,nz,faces,model", [
    (40, 18, 1, ("inlet", "outlet", "wall", "wall", "periodic", "periodic"), "bgk"),
    (40, 18, 1, ("inlet", "outlet", "wall", "wall", "periodic", "periodic"), "smagorinsky"),
    (30, 1, 9, ("inlet", "outlet", "periodic", "periodic", "wall", "freeslip"), "smagorinsky"),
    (2, 5, 4, ("inlet", "outlet", "wall", "wall", "wall", "freeslip"), "bgk"),
    (1, 1, 1, ("periodic", "periodic", "periodic", "periodic", "periodic", "periodic"), "rr3"),
])
def test_degenerate_boxes_step_by_step(nx, ny, nz, faces, model):
    """Single-layer, single-row, two-column and one-cell boxes (every
    neighbour of a cell may be itself or wrap onto one line): populations
    after 1, 2, 3, 9 and 20 steps against the oracle."""
    _say(f"degenerate box {nx}x{ny}x{nz} {model}")
    w = inputs.scaled(inputs.urban_les(), nx, ny, nz, faces=faces, model=model, tau0=0.58,
                      cs=0.1 if model != "bgk" else 0.0, inflow="uniform", ramp=3)
    solid = np.zeros((nz, ny, nx), np.uint8)
    if nx >= 30:
        solid[:, ny // 3:ny // 3 + max(1, ny // 3), 10:14] = 1 if nz == 1 else 0
        if nz > 1:
            solid[0:nz // 2, :, 10:14] = 1
    theta = (0.04, math.radians(7.0), 0.0)
    cg = sc.make_geometry(w, solid)
    ens = sc.Ensemble([cg], [[theta]])
    case = oracle_case(w, solid, theta)
    f = case.init()
    if nx * ny * nz == 1:
        # a lone periodic cell only collides: start off equilibrium
        f = f + inputs.random_populations(f.shape, 11, 2e-3)
        _, wl0, _ = orc.lattice()
        ens.f[0].view(19, cg.qs)[:, :1] = torch.from_numpy((f - wl0[:, None]).astype(np.float32)).cuda()
    _, wl, _ = orc.lattice()
    fluid = cg.fluid
    done = 0
    try:
        for target in (1, 2, 3, 9, 20):
            ens.advance(target - done)
            while done < target:
                f = case.step(done, f)
                done += 1
            g = ens.populations(0).cpu().numpy().astype(np.float64)
            ref = f - wl[:, None]
            err = np.abs(g[:, fluid] - ref[:, fluid]).max()
            scale = np.abs(ref[:, fluid]).max()
            assert err <= 1e-5 * scale + 1e-9, (target, err, scale)
    finally:
        ens.close()
