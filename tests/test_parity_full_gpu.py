"""GPU parity at the full headline size: 9x9 views of 512x512 float32, 100
hypotheses, 7x9 Census, lambda = 3, 8 paths -- the light field bench.py times,
run through lf_depth exactly as bench.py calls it.  The oracle runs the whole
method on the host (a few seconds to a few tens of seconds)."""
import numpy as np
import pytest

import lfsynth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_1907_13449_amd import lf
    oracle.build(force=False)
    lfd = lfsynth.workload("paper")
    print("full-size case:", lfd.name, flush=True)
    dev = torch.device("cuda:0")
    views = torch.from_numpy(lfd.views).to(dev)
    hyp = torch.from_numpy(lfd.hyp).to(dev)
    p = lfd.params
    ws = lf.workspace(lf.depth_workspace_bytes(lfd.S, lfd.T, lfd.H, lfd.W, lfd.N, p), dev)
    d_index = torch.empty((lfd.H, lfd.W), dtype=torch.int16, device=dev)
    disp = lf.lf_depth(views, hyp, p, ws=ws, d_index=d_index)
    ini = lf.lf_initial_disparity(views, hyp, p)
    torch.cuda.synchronize()
    g = dict(disp=disp.cpu().numpy(), d_index=d_index.cpu().numpy(),
             maps=ini["maps"].cpu().numpy(), d_init=ini["d_init"].cpu().numpy(),
             lo=ini["d_lo"].cpu().numpy(), hi=ini["d_hi"].cpu().numpy())
    o = oracle.depth(lfd.views, lfd.hyp, p, want_intermediates=True)
    return lfd, g, o


def test_full_size_initial_maps_and_bounds_bit_exact(full):
    lfd, g, o = full
    assert np.array_equal(g["maps"], o["maps"])
    assert np.array_equal(g["d_init"], o["dinit"])
    assert np.array_equal(g["lo"], o["lo"]) and np.array_equal(g["hi"], o["hi"])


def test_full_size_depth_matches_oracle(full):
    lfd, g, o = full
    assert np.array_equal(g["d_index"], o["d_index"])
    agree = float((g["disp"] == o["disparity"]).mean())
    print(f"full-size disparity agreement {agree:.6f}", flush=True)
    assert agree >= 0.999


def test_full_size_result_is_plausible(full):
    # a sanity check of the method on the synthetic ground truth, not a parity bar
    lfd, g, o = full
    err = np.abs(g["disp"] - lfd.gt)
    assert np.median(err) < 0.1
