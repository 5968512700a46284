"""lnf_filter_batch_noalloc: the batch path with its job table in the
library's static device array, for callers that cannot allocate.  Its outputs
equal lnf_filter_batch's byte for byte, on consecutive calls (the second with
fewer, smaller volumes, so stale table entries of the first would show), at
the job limit, and the size limit is refused before anything is enqueued."""
import numpy as np
import pytest

import oracle
from paper_1807_03119_amd import _lib
from paper_1807_03119_amd import phantom as ph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RULES = [(_lib.LNF_MEAN9, oracle.MEAN9), (_lib.LNF_MINVAR9, oracle.MINVAR9)]


def _jobs(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        dims = tuple(int(v) for v in rng.integers(lo, hi, 3))
        dt = np.uint8 if i % 3 == 0 else np.uint16
        kind = ["uniform", "extreme", "low"][i % 3]
        vol = torch.from_numpy(ph.random_volume(dims, dt, seed=seed * 1000 + i, kind=kind)).cuda()
        out.append((vol, int(rng.integers(1, _lib.LNF_RADIUS_MAX + 1))))
    return out


def _run(f, jobs, noalloc):
    outs = [torch.empty_like(v) for v, _ in jobs]
    triples = [(v, o, r) for (v, r), o in zip(jobs, outs)]
    if noalloc:
        rc = _lib.lnf_filter_batch_noalloc(f.handle, triples)
    else:
        rc = _lib.lnf_filter_batch(f.handle, triples)
    assert rc == _lib.LNF_OK, _lib.lnf_strerror(rc)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("rule,orule", RULES)
def test_noalloc_equals_batch_on_two_calls_in_a_row(rule, orule):
    from paper_1807_03119_amd.api import Filter
    first = _jobs(1, 40, 20, 140) + [(ph.ct_u12((300, 260, 90), seed=7, device="cuda"), 3)]
    second = _jobs(2, 6, 1, 30)
    with Filter(rule, 0) as f:
        for jobs in (first, second):
            got = _run(f, jobs, True)
            want = _run(f, jobs, False)
            for k, (a, b) in enumerate(zip(got, want)):
                assert np.array_equal(a, b), f"job {k}: {jobs[k][0].shape} r={jobs[k][1]}"
        # the small call also against the oracle
        for (v, r), a in zip(second, got):
            assert np.array_equal(a, oracle.filter_volume(v.cpu().numpy(), r, orule))


def test_noalloc_at_the_job_limit_and_beyond():
    from paper_1807_03119_amd.api import Filter
    jobs = _jobs(3, _lib.LNF_BATCH_NOALLOC_MAX, 1, 12)
    with Filter(_lib.LNF_MEAN9, 100) as f:
        got = _run(f, jobs, True)
        want = _run(f, jobs, False)
        assert all(np.array_equal(a, b) for a, b in zip(got, want))
        over = jobs + jobs[:1]
        outs = [torch.empty_like(v) for v, _ in over]
        sentinel = [o.fill_(7) for o in outs]
        rc = _lib.lnf_filter_batch_noalloc(f.handle, [(v, o, r) for (v, r), o in zip(over, outs)])
        assert rc == _lib.LNF_ERANGE
        torch.cuda.synchronize()
        assert all(bool((o == 7).all()) for o in sentinel)  # nothing ran
        assert _lib.lnf_filter_batch_noalloc(f.handle, [], 0) == _lib.LNF_OK


def test_noalloc_takes_no_device_memory():
    """After a first call (which may load the kernels), further calls leave the
    device's free memory unchanged."""
    from paper_1807_03119_amd.api import Filter
    jobs = _jobs(4, 12, 8, 60)
    with Filter(_lib.LNF_MINVAR9, 0) as f:
        _run(f, jobs, True)
        outs = [torch.empty_like(v) for v, _ in jobs]
        triples = [(v, o, r) for (v, r), o in zip(jobs, outs)]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(5):
            assert _lib.lnf_filter_batch_noalloc(f.handle, triples) == _lib.LNF_OK
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
