"""Batches and the request loop against the single-light-field path.

A batch plan runs every stage as one grouped launch over light fields of
different sizes, view counts, hypothesis counts, view types and parameters; the
request loop forms such batches from arrivals and overlaps them on the device.
Neither may change a result: every disparity map and WTA index must equal, bit
for bit, what lf_depth computes for that light field alone -- the same kernels
run the same arithmetic; only the mapping of workgroups to light fields differs.
Each output is also checked against the CPU oracle's result for that light
field with the end-to-end bar of the parity tests (at least 99.9 % of pixels
equal, for the WTA index and for the disparity)."""
import time

import numpy as np
import pytest

from cases import case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# every kernel variant: u8/f32 views, K = 1..4 hypotheses per lane, 8/16-bit
# initial path costs, 16/32-bit sums, 8/16 paths, Census cost kind, median
# on/off, 0..3 fill passes, 3-D light fields and one-row / one-column images
MIX = ["small", "f32_ragged", "u8_n65", "n256", "stage_1x11", "col_7x1", "one_row", "one_col",
       "u16_paths", "census_cost", "paths16", "paths16_u16", "boundless", "rgb_f32",
       "rgb_u8_census", "adaptive", "u8_inf_add", "fill_4", "fill_3_sparse", "u16_tail", "k3_u8",
       "k4_u16", "k3_u16", "half_shifts", "plenoptic_s", "stage_s"]


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_13449_amd import lf as binding
    return binding


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def items(lf):
    """(views, hyp, params) on the device, the alone result of each light field and
    the oracle's."""
    import oracle
    oracle.build(force=False)
    out = []
    for name in MIX:
        lfd = case(name)
        ref = oracle.depth(lfd.views, lfd.hyp, lfd.params)
        views = torch.from_numpy(np.ascontiguousarray(lfd.views)).cuda()
        hyp = torch.from_numpy(lfd.hyp).cuda()
        H, W = lfd.views.shape[-2:]
        d_index = torch.empty((H, W), dtype=torch.int16, device="cuda")
        disp = lf.lf_depth(views, hyp, lfd.params, d_index=d_index)
        torch.cuda.synchronize()
        out.append(dict(name=name, views=views, hyp=hyp, params=lfd.params,
                        disp=disp.cpu().numpy(), d_index=d_index.cpu().numpy(),
                        oracle_disp=ref["disparity"], oracle_index=ref["d_index"]))
    return out


def _outputs(items, order):
    res = []
    for i in order:
        it = items[i]
        H, W = it["disp"].shape
        res.append((torch.full((H, W), float("nan"), device="cuda"),
                    torch.full((H, W), -7, dtype=torch.int16, device="cuda")))
    return res


def _plan(lf, items, order, outs, tuning=None):
    return lf.Plan([(items[i]["views"], items[i]["hyp"], items[i]["params"], o[0], o[1])
                    for i, o in zip(order, outs)], tuning=tuning)


def _check(items, order, outs):
    for i, (disp, d_index) in zip(order, outs):
        it = items[i]
        got_d, got_i = disp.cpu().numpy(), d_index.cpu().numpy()
        assert np.array_equal(got_d, it["disp"]), it["name"]
        assert np.array_equal(got_i, it["d_index"]), it["name"]
        # and against the oracle, with the end-to-end bar of the parity tests
        assert (got_i == it["oracle_index"]).mean() >= 0.999, it["name"]
        assert (got_d == it["oracle_disp"]).mean() >= 0.999, it["name"]


def test_batch_equals_alone(lf, items):
    order = list(range(len(items)))
    outs = _outputs(items, order)
    say("batch of", len(order))
    plan = _plan(lf, items, order, outs)
    plan.run()
    torch.cuda.synchronize()
    _check(items, order, outs)
    # one grouped launch per stage and kernel variant, not one per light field
    assert plan.launches < 10 * len(order)


@pytest.mark.parametrize("tuning", [
    dict(cost_cells_per_thread=2, dense_prefetch=4, bounded_prefetch=4, bounded_lanes=64),
    dict(cost_cells_per_thread=8, cost_stride=4, dense_prefetch=16, bounded_prefetch=8,
         bounded_lanes=64),
    dict(bounded_prefetch=16, bounded_offsets=64),    # the 64-bit addressed bounded SGM
    dict(cost_cells_per_thread=4, cost_stride=2, dense_prefetch=8, bounded_lanes=32),
    dict(bounded_lanes=16),
])
def test_batch_every_tuning(lf, items, tuning):
    order = [3, 0, 1, 1, 9, 2, 10, 25, 23, 13]       # repeats and a shuffled order
    outs = _outputs(items, order)
    say("tuning", tuning)
    plan = _plan(lf, items, order, outs, tuning)
    plan.run()
    torch.cuda.synchronize()
    _check(items, order, outs)


def test_single_path_tuning_independent(lf, items):
    # the single-light-field path at default tuning equals a batch of one at another
    outs = _outputs(items, [1])
    plan = _plan(lf, items, [1], outs, dict(cost_cells_per_thread=4, cost_stride=4))
    plan.run()
    torch.cuda.synchronize()
    _check(items, [1], outs)


def test_graph_replays(lf, items):
    order = list(range(len(items)))
    outs = _outputs(items, order)
    plan = _plan(lf, items, order, outs)
    torch.cuda.synchronize()
    plan.capture()
    for rep in range(3):
        for d, x in outs:                            # eager work between the replays
            d.fill_(float("nan"))
            x.fill_(-7)
        torch.cuda.synchronize()
        say("replay", rep)
        plan.run()
        torch.cuda.synchronize()
        _check(items, order, outs)


def test_autotune_keeps_results(lf, items):
    order = [0, 1, 4, 8]
    outs = _outputs(items, order)
    plan = _plan(lf, items, order, outs)
    chosen = plan.autotune(reps=1)
    say("autotune chose", chosen)
    assert chosen["cost_cells_per_thread"] in (2, 4, 8)
    assert chosen["cost_stride"] in (1, 2, 4)
    assert chosen["dense_prefetch"] in (4, 8, 16)
    assert chosen["bounded_prefetch"] in (4, 8, 16)
    assert chosen["bounded_lanes"] in (16, 32, 64)
    assert plan.tuning == chosen
    torch.cuda.synchronize()
    _check(items, order, outs)
    for d, x in outs:
        d.fill_(float("nan"))
    plan.capture()
    plan.run()
    torch.cuda.synchronize()
    _check(items, order, outs)


def _serve(lf, items, order, arena_bytes, max_batch, max_inflight, gaps):
    srv = lf.Server(arena_bytes, "cuda", max_batch=max_batch, max_inflight=max_inflight)
    outs = _outputs(items, order)
    torch.cuda.synchronize()
    tickets = []
    for i, o, gap in zip(order, outs, gaps):
        it = items[i]
        tickets.append(srv.submit(it["views"], it["hyp"], it["params"], o[0], o[1]))
        if gap:
            time.sleep(gap)
    infos = [srv.wait(t, timeout=60.0) for t in tickets]
    stats = srv.stats()
    srv.close()
    return outs, infos, stats


def test_served_equals_alone(lf, items):
    rng = np.random.default_rng(5)
    order = list(rng.integers(0, len(items), size=24))
    gaps = rng.exponential(0.002, size=len(order))     # arrivals while others run
    outs, infos, stats = _serve(lf, items, order, 1 << 30, 4, 2, gaps)
    say("served", stats, "batches sizes", sorted({(i["batch"], i["batch_size"]) for i in infos}))
    for inf in infos:
        assert inf["status"] == 0, inf
        assert inf["t_submit"] <= inf["t_admit"] <= inf["t_launch"] <= inf["t_done"]
    _check(items, order, outs)
    assert stats["completed"] == len(order)
    assert stats["arena_in_use"] == 0
    assert stats["arena_peak"] <= 1 << 30


def test_served_waits_for_the_submitting_stream(lf, items):
    # the inputs and outputs are written by kernels still queued on torch's stream
    # when the request is submitted (no synchronisation in between): the server's
    # stream must wait for them
    srv = lf.Server(1 << 30, "cuda", max_batch=4, max_inflight=2)
    order = [0, 1, 2, 1]
    outs = _outputs(items, order)
    torch.cuda.synchronize()
    tickets = []
    for i, o in zip(order, outs):
        it = items[i]
        big = torch.empty((1 << 26,), device="cuda")
        big.normal_()                                # keeps the stream busy for a while
        views = it["views"].clone()                  # produced on the stream, not yet done
        hyp = it["hyp"].clone()
        o[0].fill_(float("nan"))
        o[1].fill_(-7)
        tickets.append((srv.submit(views, hyp, it["params"], o[0], o[1]), views, hyp, big))
    infos = [srv.wait(t[0], timeout=60.0) for t in tickets]
    srv.close()
    assert all(inf["status"] == 0 for inf in infos)
    torch.cuda.synchronize()
    _check(items, order, outs)


def test_served_under_a_tight_arena(lf, items):
    # an arena that fits the largest request alone: admission serialises the
    # large ones and still packs small ones beside them
    order = [1, 0, 1, 4, 8, 1, 0]
    need = max(lf.batch_workspace_bytes([lf.make_request(items[i]["views"], items[i]["hyp"],
                                                         items[i]["params"], torch.empty(
                                                             items[i]["disp"].shape,
                                                             device="cuda"))]) for i in order)
    outs, infos, stats = _serve(lf, items, order, need, 8, 2, [0.0] * len(order))
    say("tight arena", need, stats)
    assert all(inf["status"] == 0 for inf in infos)
    assert stats["arena_peak"] <= need
    _check(items, order, outs)
