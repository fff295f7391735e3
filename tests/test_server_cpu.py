"""Host-side behaviour of the batch plan and the request loop, without a GPU:
argument checks, admission limits, and failure handling when the device cannot
be used (here: there is none, so every launch attempt fails and each request
must complete with LF_EDEVICE, its memory returned, the loop still serving)."""
import ctypes as C

import numpy as np
import pytest


@pytest.fixture(scope="module")
def lf():
    from paper_1907_13449_amd import lf as binding
    return binding


FAKE = 1 << 20            # an aligned address that is never dereferenced here


def _req(lf, S=5, T=5, H=32, W=40, N=16, data=FAKE, dtype=1, **prm):
    import lfsynth
    p = lfsynth._params(census=(5, 5), p_init=(10, 120), p_final=(10, 120), lam=2,
                        edge_tau=float("inf"), alpha=255.0, sum_bits=32)
    p.update(prm)
    vs = lf.ViewSet(data, S, T, H, W, W, dtype, 1)
    return lf.Request(vs, FAKE, N, lf.make_params(p), FAKE, 0)


def _cfg(lf, arena=FAKE, nbytes=1 << 30, max_batch=4, max_inflight=2, max_queue=64, ratio=0,
         large=0, max_large=0):
    return lf.ServerConfig(arena, nbytes, max_batch, max_inflight, max_queue, ratio, lf.Tuning(),
                           large, max_large)


def _create(lf, cfg):
    h = C.c_void_p()
    st = lf.lib.lf_server_create(C.byref(cfg), C.byref(h))
    return st, h


def test_batch_workspace_is_the_sum_plus_tables(lf):
    a, b = _req(lf), _req(lf, H=50, W=21, N=40)
    one_a = lf.batch_workspace_bytes([a])
    one_b = lf.batch_workspace_bytes([b])
    both = lf.batch_workspace_bytes([a, b])
    da = lf.lib.lf_depth_workspace_size(5, 5, 1, 32, 40, 16, C.byref(a.params))
    db = lf.lib.lf_depth_workspace_size(5, 5, 1, 50, 21, 40, C.byref(b.params))
    assert one_a > da and one_b > db
    # the batch holds both members' workspaces and one set of tables
    assert both >= one_a + db - 1 and both >= one_b + da - 1
    assert both < one_a + one_b
    bad = _req(lf, S=4)
    assert lf.batch_workspace_bytes([a, bad]) == 0


def test_plan_create_rejects_bad_input(lf):
    reqs = (lf.Request * 2)(_req(lf), _req(lf, N=1))
    h = C.c_void_p()
    st = lf.lib.lf_plan_create(reqs, 2, C.c_void_p(FAKE), 1 << 30, None, None, C.byref(h))
    assert st == lf.LF_EINVAL and not h.value
    reqs = (lf.Request * 1)(_req(lf))
    st = lf.lib.lf_plan_create(reqs, 1, C.c_void_p(FAKE + 8), 1 << 30, None, None, C.byref(h))
    assert st == lf.LF_EINVAL                      # unaligned workspace
    st = lf.lib.lf_plan_create(reqs, 1, C.c_void_p(FAKE), 1024, None, None, C.byref(h))
    assert st == lf.LF_ENOSPACE
    for t in (lf.Tuning(3, 0, 0, 0),               # 3 cells per thread is not offered
              lf.Tuning(0, 0, 0, 0, 0, 48)):       # nor 48-bit offsets
        st = lf.lib.lf_plan_create(reqs, 1, C.c_void_p(FAKE), 1 << 30, C.byref(t), None,
                                   C.byref(h))
        assert st == lf.LF_EINVAL
        assert "tuning" in lf.lib.lf_last_error().decode()


def test_server_config_checks(lf):
    for cfg in (_cfg(lf, arena=0), _cfg(lf, arena=FAKE + 8), _cfg(lf, max_batch=0),
                _cfg(lf, max_inflight=5), _cfg(lf, max_queue=0), _cfg(lf, ratio=1),
                _cfg(lf, large=-1), _cfg(lf, max_large=-1), _cfg(lf, max_large=5),
                _cfg(lf, ratio=-2)):
        st, h = _create(lf, cfg)
        assert st == lf.LF_EINVAL and not h.value


def test_submit_checks_and_admission_limit(lf):
    st, h = _create(lf, _cfg(lf, nbytes=64 << 20))
    assert st == lf.LF_OK
    try:
        tk = C.c_int64()
        assert lf.lib.lf_server_submit(h, C.byref(_req(lf, N=300)), None, C.byref(tk)) == lf.LF_EUNSUPPORTED
        assert lf.lib.lf_server_submit(h, C.byref(_req(lf, data=0)), None, C.byref(tk)) == lf.LF_EINVAL
        # a light field whose workspace can never fit in the arena is refused at once
        big = _req(lf, S=9, T=9, H=512, W=512, N=100)
        assert lf.lib.lf_server_submit(h, C.byref(big), None, C.byref(tk)) == lf.LF_ENOSPACE
        assert "arena" in lf.lib.lf_last_error().decode()
        info = lf.RequestInfo()
        assert lf.lib.lf_server_wait(h, 12345, 0.0, C.byref(info)) == lf.LF_EINVAL
    finally:
        lf.lib.lf_server_destroy(h)


def test_device_failure_completes_requests_with_an_error(lf):
    # no GPU here: creating the server's streams fails, so every batch fails; each
    # request must still complete (LF_EDEVICE), give its memory back, and the loop
    # must keep taking requests
    st, h = _create(lf, _cfg(lf))
    assert st == lf.LF_OK
    try:
        tickets = []
        for i in range(6):
            tk = C.c_int64()
            assert lf.lib.lf_server_submit(h, C.byref(_req(lf, N=8 + i)), None, C.byref(tk)) == lf.LF_OK
            tickets.append(tk.value)
        for t in tickets:
            info = lf.RequestInfo()
            st = lf.lib.lf_server_wait(h, t, 30.0, C.byref(info))
            assert st == lf.LF_EDEVICE, (st, lf.lib.lf_last_error())
            assert info.status == lf.LF_EDEVICE
            assert info.t_submit <= info.t_admit <= info.t_done
        v = [C.c_int64() for _ in range(4)]
        lf.lib.lf_server_stats(h, *[C.byref(x) for x in v])
        assert v[0].value == 6                     # completed
        assert v[2].value == 0                     # arena in use
        assert lf.lib.lf_server_wait(h, tickets[0], 0.0, None) == lf.LF_EINVAL   # forgotten
    finally:
        lf.lib.lf_server_destroy(h)


def test_destroy_cancels_queued_requests(lf):
    st, h = _create(lf, _cfg(lf, max_queue=512))
    assert st == lf.LF_OK
    for _ in range(200):
        tk = C.c_int64()
        assert lf.lib.lf_server_submit(h, C.byref(_req(lf)), None, C.byref(tk)) == lf.LF_OK
    lf.lib.lf_server_destroy(h)                    # returns: nothing is left waiting


def test_queue_limit(lf):
    # submissions beyond max_queue pending requests are refused with LF_EBUSY
    st, h = _create(lf, _cfg(lf, max_queue=1))
    assert st == lf.LF_OK
    try:
        codes = set()
        for _ in range(400):
            tk = C.c_int64()
            codes.add(lf.lib.lf_server_submit(h, C.byref(_req(lf)), None, C.byref(tk)))
        assert codes <= {lf.LF_OK, lf.LF_EBUSY}
        assert lf.LF_OK in codes
    finally:
        lf.lib.lf_server_destroy(h)
