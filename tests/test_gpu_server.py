"""Request server: results identical alone and in the mix, admission under the
memory cap with LRU eviction, failure isolation, cancellation, FIFO mode.
Failure paths are forced from the host (a batch fails before launch); no
test makes the GPU fault."""
import numpy as np
import pytest

import oracle
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pinned(arr):
    t = torch.empty(arr.shape, dtype=torch.uint8 if arr.dtype == np.uint8 else torch.uint16,
                    pin_memory=True)
    t.numpy()[...] = arr
    return t


def _empty_pinned_like(t):
    return torch.empty(t.shape, dtype=t.dtype, pin_memory=True)


def _filter(rule=_lib.LNF_MEAN9, gate=0):
    from paper_1807_03119_amd.api import Filter
    return Filter(rule, gate)


def _server(f, **kw):
    from paper_1807_03119_amd.api import Server
    return Server(f, **kw)


def _volumes(n, seed):
    rng = np.random.default_rng(seed)
    vols = []
    for i in range(n):
        dims = tuple(int(v) for v in rng.integers(8, 48, 3))
        vols.append(ph.small_u8(seed + i, dims=dims) if i % 2 == 0
                    else ph.ct_u12(dims, seed=seed + i))
    return vols


@pytest.mark.parametrize("mode", [_lib.LNF_SERVE_BATCHED, _lib.LNF_SERVE_FIFO])
def test_results_same_alone_and_in_the_mix(mode):
    vols = _volumes(6, 300)
    rng = np.random.default_rng(1)
    with _filter() as f, _server(f, mode=mode, n_streams=3, max_batch=8) as s:
        ids = []
        for v in vols:
            rc, vid = s.put(_pinned(v))
            assert rc == 0
            ids.append(vid)
        reqs = []
        for k in range(24):  # several requests per volume, mixed radii
            i = int(rng.integers(0, len(vols)))
            r = int(rng.integers(1, 5))
            out = torch.empty(vols[i].shape, dtype=torch.uint8 if vols[i].dtype == np.uint8
                              else torch.uint16, pin_memory=True)
            rc, t = s.submit(ids[i], r, host_out=out)
            assert rc == 0
            reqs.append((t, i, r, out))
        for t, i, r, out in reqs:
            assert s.wait(t, 60000) == 0
            alone = f(torch.from_numpy(vols[i]).cuda(), r).cpu().numpy()
            np.testing.assert_array_equal(out.numpy(), alone)
            np.testing.assert_array_equal(out.numpy(), oracle.filter_volume(vols[i], r))
        st = s.stats()
        assert st["completed"] == 24 and st["failed"] == 0
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
        if mode == _lib.LNF_SERVE_FIFO:
            assert st["batches"] == 24


def test_admission_cap_evicts_idle_volumes_lru():
    vol = ph.ct_u12((64, 64, 64), seed=7)  # 512 KiB each
    cap = 3 << 20
    with _filter() as f, _server(f, cap_bytes=cap, max_batch=4) as s:
        host = _pinned(vol)
        ids = []
        for _ in range(12):
            rc, vid = s.put(host)
            assert rc == 0
            ids.append(vid)
        s.sync()
        st = s.stats()
        assert st["evictions"] > 0 and st["peak_bytes"] <= cap
        # the oldest volumes were evicted, the newest are resident
        rc, _ = s.submit(ids[0], 1)
        assert rc == _lib.LNF_ENOTFOUND
        out = _empty_pinned_like(host)
        rc, t = s.submit(ids[-1], 2, host_out=out)
        assert rc == 0 and s.wait(t, 60000) == 0
        np.testing.assert_array_equal(out.numpy(), oracle.filter_volume(vol, 2))
        # a volume larger than the whole cap is refused
        big = torch.empty((64, 128, 256), dtype=torch.uint16, pin_memory=True)
        rc, _ = s.put(big)
        assert rc == _lib.LNF_EBUSY
        assert s.stats()["peak_bytes"] <= cap


def test_failed_batch_fails_only_its_requests():
    vols = _volumes(3, 500)
    with _filter() as f, _server(f, max_batch=1, fail_batch=2) as s:
        ids = [s.put(_pinned(v))[1] for v in vols]
        outs, tickets = [], []
        for k in range(5):
            i = k % 3
            out = torch.empty(vols[i].shape, dtype=torch.uint8 if vols[i].dtype == np.uint8
                              else torch.uint16, pin_memory=True)
            rc, t = s.submit(ids[i], 1, host_out=out)
            assert rc == 0
            assert s.wait(t, 60000) in (0, _lib.LNF_ECANCELED)  # serialise: batch k+1 = request k
            outs.append((i, out))
            tickets.append(t)
        codes = [s.poll(t)[0] for t in tickets]
        assert codes == [0, _lib.LNF_ECANCELED, 0, 0, 0]
        for (i, out), c in zip(outs, codes):
            if c == 0:
                np.testing.assert_array_equal(out.numpy(), oracle.filter_volume(vols[i], 1))
        st = s.stats()
        assert st["failed"] == 1 and st["completed"] == 4


def test_cancel_release_and_bad_arguments():
    vol = ph.small_u8(9, dims=(16, 16, 16))
    with _filter() as f, _server(f) as s:
        rc, vid = s.put(_pinned(vol))
        assert rc == 0
        rc, t = s.submit(vid, 3)
        assert rc == 0 and s.wait(t, 60000) == 0
        assert s.cancel(t) == _lib.LNF_EBUSY          # already done
        assert s.cancel(10 ** 9) == _lib.LNF_ENOTFOUND
        assert s.submit(vid, 0)[0] == _lib.LNF_EINVAL
        assert s.submit(vid + 999, 1)[0] == _lib.LNF_ENOTFOUND
        assert s.release(vid) == 0
        assert s.release(vid) == _lib.LNF_ENOTFOUND
        assert s.submit(vid, 1)[0] == _lib.LNF_ENOTFOUND
        assert s.wait(10 ** 9, 10) == _lib.LNF_ENOTFOUND


def test_pitched_upload_of_a_crop():
    big = ph.ct_u12((40, 30, 20), seed=11)
    host = _pinned(big)
    crop = np.ascontiguousarray(big[3:15, 5:25, 7:33])  # nz=12, ny=20, nx=26
    with _filter() as f, _server(f) as s:
        ptr = host.data_ptr() + (3 * 30 * 40 + 5 * 40 + 7) * 2
        rc, vid = s.put(ptr, dims=(26, 20, 12), dtype=_lib.LNF_U16, pitch=(40, 40 * 30))
        assert rc == 0
        out = torch.empty(crop.shape, dtype=torch.uint16, pin_memory=True)
        rc, t = s.submit(vid, 2, host_out=out)
        assert rc == 0 and s.wait(t, 60000) == 0
        np.testing.assert_array_equal(out.numpy(), oracle.filter_volume(crop, 2))


def test_continuous_batching_groups_requests():
    vols = _volumes(4, 700)
    with _filter() as f, _server(f, n_streams=2, max_batch=64) as s:
        ids = [s.put(_pinned(v))[1] for v in vols]
        s.sync()
        tickets = [s.submit(ids[k % 4], 1 + k % 3)[1] for k in range(40)]
        for t in tickets:
            assert s.wait(t, 60000) == 0
        st = s.stats()
        assert st["completed"] == 40
        assert st["batches"] < 40  # requests that queued up were launched together


def test_requests_that_cannot_fit_end_with_ebusy():
    """A volume whose output would not fit beside it under the cap is refused at
    submit; requests whose own volumes fill the cap end with LNF_EBUSY instead
    of waiting forever (the queue moves on and sync returns)."""
    import threading
    cap = 3 << 20
    with _filter() as f, _server(f, cap_bytes=cap, max_batch=4) as s:
        big = ph.ct_u12((128, 128, 64), seed=21)            # 2 MiB: 2 + 2 > 3 MiB
        rc, vid = s.put(_pinned(big))
        assert rc == 0
        assert s.submit(vid, 1)[0] == _lib.LNF_EBUSY
        assert s.release(vid) == 0
        half = ph.ct_u12((128, 96, 64), seed=22)            # 1.5 MiB each: both fill the cap
        rc_a, a = s.put(_pinned(half))
        rc_b, b = s.put(_pinned(half))
        assert rc_a == 0 and rc_b == 0
        tickets = []
        for vid in (a, b):
            rc, t = s.submit(vid, 1)
            assert rc in (0, _lib.LNF_ENOTFOUND)            # b may already be evicted
            if rc == 0:
                tickets.append(t)
        done = threading.Event()
        threading.Thread(target=lambda: (s.sync(), done.set()), daemon=True).start()
        assert done.wait(30), "server sync did not return"
        for t in tickets:
            assert s.wait(t, 1000) in (0, _lib.LNF_EBUSY)
        assert s.stats()["peak_bytes"] <= cap


def test_cancel_wakes_a_waiting_thread():
    """lnf_server_wait on a ticket returns as soon as another thread cancels it."""
    import threading
    import time
    # requests that take longer to run than to submit, so the queue builds up
    vol = np.random.default_rng(23).integers(0, 4096, (256, 256, 256), dtype=np.uint16)
    with _filter() as f, _server(f, mode=_lib.LNF_SERVE_FIFO) as s:
        rc, vid = s.put(_pinned(vol))
        assert rc == 0
        for attempt in range(5):
            tickets = [s.submit(vid, 4)[1] for _ in range(96)]
            last = tickets[-1]
            res = {}
            th = threading.Thread(target=lambda: res.setdefault("rc", s.wait(last, -1)), daemon=True)
            th.start()
            time.sleep(0.001)
            rc = s.cancel(last)
            th.join(20)
            assert not th.is_alive(), "waiter not woken"
            s.sync()
            if rc == 0:
                assert res["rc"] == _lib.LNF_ECANCELED
                return
            assert rc == _lib.LNF_EBUSY and res["rc"] == 0  # it had already started
        pytest.skip("the request always started before it could be cancelled")


def test_micro_batches_keep_the_voxel_budget():
    """With a budget of 2^20 voxels, requests on 96^3 volumes (884,736 voxels)
    can never share a micro-batch, and 32^3 ones at most 32 to a batch."""
    big = ph.ct_u12((96, 96, 96), seed=31)
    small = ph.ct_u12((32, 32, 32), seed=32)
    with _filter() as f, _server(f, max_batch=256, batch_mvox=1) as s:
        rc_b, vb = s.put(_pinned(big))
        rc_s, vs = s.put(_pinned(small))
        assert rc_b == 0 and rc_s == 0
        s.sync()
        s.stats(reset=True)
        n = 12
        tickets = [s.submit(vb, 1 + k % 3)[1] for k in range(n)]
        s.sync()
        assert all(s.wait(t, 1000) == 0 for t in tickets)
        assert s.stats(reset=True)["batches"] == n
        tickets = [s.submit(vs, 1 + k % 3)[1] for k in range(200)]
        s.sync()
        assert all(s.wait(t, 1000) == 0 for t in tickets)
        assert s.stats()["batches"] >= -(-200 // 32)
    with _filter() as f:
        with pytest.raises(_lib.LnfError):
            _server(f, batch_mvox=-1)


@pytest.mark.timeout(600)
def test_results_same_alone_and_in_the_mix_large_volumes():
    """Benchmark-sized volumes (sides 128..512) through the batched server with
    mixed radii and both voxel types: every output equals the volume filtered
    alone, and sampled voxels equal the oracle."""
    rng = np.random.default_rng(41)
    dims = [(128, 128, 128), (200, 160, 144), (320, 256, 192), (512, 512, 512), (250, 130, 170)]
    vols = [ph.ct_u12(d, seed=4100 + i, device="cuda").cpu().numpy() if i != 4
            else ph.small_u8(4104, dims=d) for i, d in enumerate(dims)]
    with _filter() as f, _server(f, n_streams=4, max_batch=64) as s:
        ids = []
        for v in vols:
            rc, vid = s.put(_pinned(v))
            assert rc == 0
            ids.append(vid)
        reqs = []
        for k in range(14):
            i = k % len(vols) if k < len(vols) else int(rng.integers(0, len(vols)))
            r = int(rng.integers(1, 4))
            out = _empty_pinned_like(torch.from_numpy(vols[i]))
            rc, t = s.submit(ids[i], r, host_out=out)
            assert rc == 0
            reqs.append((t, i, r, out))
        for t, i, r, out in reqs:
            assert s.wait(t, 120000) == 0
            got = out.numpy()
            alone = f(torch.from_numpy(vols[i]).cuda(), r).cpu().numpy()
            assert np.array_equal(got, alone), f"volume {dims[i]} r={r}"
            nz, ny, nx = vols[i].shape
            pts = np.stack([rng.integers(0, nx, 400), rng.integers(0, ny, 400),
                            rng.integers(0, nz, 400)], 1)
            pts[:8] = [[0, 0, 0], [nx - 1, ny - 1, nz - 1], [0, ny - 1, 0], [nx - 1, 0, nz - 1],
                       [nx // 2, 0, nz // 2], [0, ny // 2, nz - 1], [nx - 1, ny // 2, 0],
                       [nx // 2, ny // 2, nz // 2]]
            want = oracle.filter_points(vols[i], r, pts)
            assert np.array_equal(got[pts[:, 2], pts[:, 1], pts[:, 0]].astype(np.uint32), want)
        assert s.stats()["completed"] == 14
