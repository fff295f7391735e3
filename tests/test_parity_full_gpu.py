"""GPU parity at full workload sizes, through lf_depth exactly as bench.py calls
it, against the oracle running the whole method on the host.

  - the benchmark light field: 9x9 views of 512x512 float32, 100 hypotheses, 7x9
    Census, lambda = 3, 8 paths (a few seconds of oracle time);
  - slow: the two shapes of the large workload -- 15x15 plenoptic-like views of
    625x434 float32 (N = 64, d in [-1.5, 1.5]) and an 1x11 moving-stage light
    field of 1920x1080 uint8 (N = 96, d in [0, 24], two cross views, shifts up to
    120 px) -- tens of seconds of oracle time each.

Bars as in the reduced-size parity tests: the initial stage (Census cost volume
and aggregated cost of every cross view, D_i, d_init, bounds) and the final WTA
index bit-exact; the disparity on at least 99.9 % of pixels."""
import numpy as np
import pytest

import lfsynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_1907_13449_amd import lf
    oracle.build(force=False)
    lfd = lfsynth.workload(name)
    print("full-size case:", lfd.name, flush=True)
    dev = torch.device("cuda:0")
    views = torch.from_numpy(lfd.views).to(dev)
    hyp = torch.from_numpy(lfd.hyp).to(dev)
    p = lfd.params
    ws = lf.workspace(lf.depth_workspace_bytes(lfd.S, lfd.T, lfd.H, lfd.W, lfd.N, p), dev)
    d_index = torch.empty((lfd.H, lfd.W), dtype=torch.int16, device=dev)
    disp = lf.lf_depth(views, hyp, p, ws=ws, d_index=d_index)
    torch.cuda.synchronize()
    del ws
    ini = lf.lf_initial_disparity(views, hyp, p, want_volumes=True)
    torch.cuda.synchronize()
    g = dict(disp=disp.cpu().numpy(), d_index=d_index.cpu().numpy(),
             maps=ini["maps"].cpu().numpy(), d_init=ini["d_init"].cpu().numpy(),
             lo=ini["d_lo"].cpu().numpy(), hi=ini["d_hi"].cpu().numpy())
    ccv = ini["census_cost"].cpu().numpy()
    csum = ini["csum_init"].cpu().numpy().view(np.uint16)
    del ini
    torch.cuda.empty_cache()
    print("  GPU done; oracle running", flush=True)
    o = oracle.depth(lfd.views, lfd.hyp, p, want_intermediates=True, want_initial_volumes=True)
    print("  oracle done", flush=True)
    # compared here, and only the outcomes kept (several GB at the largest shape)
    g["init_cost_equal"] = bool(np.array_equal(ccv, o.pop("init_cost")))
    g["init_csum_equal"] = bool(np.array_equal(csum, o.pop("init_csum")))
    del ccv, csum
    for k in ("cost", "csum"):
        o.pop(k)
    return lfd, g, o


def _check(lfd, g, o):
    assert g["init_cost_equal"]
    assert g["init_csum_equal"]
    assert np.array_equal(g["maps"], o["maps"])
    assert np.array_equal(g["d_init"], o["dinit"])
    assert np.array_equal(g["lo"], o["lo"]) and np.array_equal(g["hi"], o["hi"])
    assert np.array_equal(g["d_index"], o["d_index"])
    agree = float((g["disp"] == o["disparity"]).mean())
    print(f"{lfd.name}: disparity agreement {agree:.6f}", flush=True)
    assert agree >= 0.999


@pytest.fixture(scope="module")
def full():
    return _run("paper")


def test_full_size_initial_stage_bit_exact(full):
    lfd, g, o = full
    assert g["init_cost_equal"]
    assert g["init_csum_equal"]
    assert np.array_equal(g["maps"], o["maps"])
    assert np.array_equal(g["d_init"], o["dinit"])
    assert np.array_equal(g["lo"], o["lo"]) and np.array_equal(g["hi"], o["hi"])


def test_full_size_depth_matches_oracle(full):
    _check(*full)


def test_full_size_result_is_plausible(full):
    # a sanity check of the method on the synthetic ground truth, not a parity bar
    lfd, g, o = full
    err = np.abs(g["disp"] - lfd.gt)
    assert np.median(err) < 0.1


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_full_size_plenoptic_15x15_matches_oracle():
    _check(*_run("plenoptic"))


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_full_size_moving_stage_1x11_matches_oracle():
    _check(*_run("stage"))
