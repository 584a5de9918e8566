"""The request loop on the GPU: results, admission, cancellation (needs an MI355X)."""
import sys
import threading
import time

import numpy as np
import pytest

from paper_1005_5198_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1005_5198_amd as rs_mod
    return rs_mod


def small_requests(n, seed=40):
    children = np.random.SeedSequence(seed).spawn(n)
    return [w.random_map(np.random.default_rng(c), f"req{k}", rays_per_px=8.0, src_choices=(128, 256))
            for k, c in enumerate(children)]


def test_served_maps_equal_alone(rs):
    specs = small_requests(10)
    with rs.Server(hbm_budget_bytes=256 << 20, max_inflight=4, mode="mixed", slice_ms=2.0) as srv:
        tickets = []
        for k, s in enumerate(specs):
            tickets.append(srv.submit(s.params, s.lens_xy, s.lens_m))
            if k % 3 == 0:
                time.sleep(0.002)
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    say("server stats", st)
    assert st["completed"] == len(specs) and st["failed"] == 0 and st["hbm_in_use_bytes"] == 0
    assert st["steps"] >= 1 and st["latency_p99_s"] >= st["latency_p50_s"] > 0
    for s, (m, stats, lat) in zip(specs, results):
        alone, st1 = rs.make_map(s.params, s.lens_xy, s.lens_m, mode="mixed", return_stats=True)
        assert np.array_equal(m, alone.cpu().numpy()), s.name
        for key in ("rays_shot", "rays_in_map", "rays_out", "rays_singular"):
            assert stats[key] == st1[key], (s.name, key)
        assert lat > 0


def test_budget_makes_requests_wait(rs):
    """A pool that holds one request at a time still serves all of them, in order."""
    specs = small_requests(4, seed=41)
    one = max(16 * s.n_lens + 4 * s.params["npx"] * s.params["npy"] for s in specs) + 4096
    with rs.Server(hbm_budget_bytes=int(one * 1.5), max_inflight=8, mode="mixed", slice_ms=2.0) as srv:
        tickets = [srv.submit(s.params, s.lens_xy) for s in specs]
        maps = [srv.wait(t)[0] for t in tickets]
        st = srv.stats()
    say("budget stats", st)
    assert st["completed"] == 4 and st["hbm_peak_bytes"] <= int(one * 1.5)
    assert st["max_waiting"] >= 1
    for s, m in zip(specs, maps):
        assert np.array_equal(m, rs.make_map(s.params, s.lens_xy, mode="mixed").cpu().numpy())


def test_cancel_and_oversize(rs):
    from paper_1005_5198_amd._lib import RayshootError, RS_ECANCELED, RS_ENOMEM
    big = w.config2().window(0, 19200, 0, 1024)          # ~3.4e11 interactions, long enough to cancel
    small = small_requests(2, seed=42)
    with rs.Server(hbm_budget_bytes=64 << 20, max_inflight=4, mode="mixed", slice_ms=5.0) as srv:
        tb = srv.submit(big.params, big.lens_xy)
        ts = [srv.submit(s.params, s.lens_xy) for s in small]
        srv.cancel(tb)
        with pytest.raises(RayshootError) as e:
            srv.wait(tb)
        assert e.value.code == RS_ECANCELED
        for s, t in zip(small, ts):
            m, _, _ = srv.wait(t)
            assert np.array_equal(m, rs.make_map(s.params, s.lens_xy, mode="mixed").cpu().numpy())
        huge = w.make_params(0.3, 0.0, 0.0, (-1.0, -1.0, 2.0, 2.0, 64, 64), (-1.0, -1.0, 2.0, 2.0, 8192, 8192))
        th = srv.submit(huge, np.zeros((0, 2)))
        with pytest.raises(RayshootError) as e:
            srv.wait(th)
        assert e.value.code == RS_ENOMEM
        st = srv.stats()
    assert st["canceled"] == 1 and st["failed"] == 1 and st["completed"] == 2


def test_full_queue_refuses_with_ebusy(rs):
    """One slot, a waiting queue of two: a burst of submissions behind a long request is
    refused with RS_EBUSY beyond the queue; the accepted ones equal maps made alone."""
    from paper_1005_5198_amd._lib import RayshootError, RS_EBUSY
    long_one = w.config2().window(0, 19200, 0, 640)        # ~2e11 interactions, tens of ms
    small = small_requests(6, seed=43)
    with rs.Server(hbm_budget_bytes=256 << 20, max_inflight=1, mode="mixed", slice_ms=5.0, max_waiting=2) as srv:
        accepted = [(long_one, srv.submit(long_one.params, long_one.lens_xy))]
        refused = 0
        for s in small:
            try:
                accepted.append((s, srv.submit(s.params, s.lens_xy)))
            except RayshootError as e:
                assert e.code == RS_EBUSY
                refused += 1
        maps = [(s, srv.wait(t)[0]) for s, t in accepted]
        st = srv.stats()
    say("ebusy stats", st, "refused", refused)
    assert refused >= 1 and st["rejected_busy"] == refused
    assert st["completed"] == len(accepted)
    for s, m in maps:
        assert np.array_equal(m, rs.make_map(s.params, s.lens_xy, mode="mixed").cpu().numpy()), s.name
