"""wpm_enumerate_noalloc (the entry point for callers that cannot allocate)
against wpm_enumerate, through the C ABI: two calls in a row, the second on
a smaller batch, each compared with the allocating entry point's counts,
totals and records (bit-exact, records as multisets)."""
import ctypes
import sys

import numpy as np
import pytest

import wpm_inputs as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(E, L, batch, items, fn, use_scratch):
    """One call of `fn` (wpm_enumerate or wpm_enumerate_noalloc) on fresh
    output buffers -> (counts, totals, sorted used records)."""
    n = len(batch.preps)
    cap = 1 << 20
    surv = torch.full((cap, 2), 7, dtype=torch.int64, device="cuda")
    counts = torch.full((n,), 7, dtype=torch.int64, device="cuda")
    total = torch.full((L.TOTAL_WORDS,), 7, dtype=torch.int64, device="cuda")
    scratch = torch.full((4,), 7, dtype=torch.int64, device="cuda")
    d_items = torch.from_numpy(items.view(np.int64).reshape(-1).copy()).to("cuda")
    s = L.Sched(mode=L.SCHED_DYNAMIC, wg_size=128, grid=0, flags=0, d_items=d_items.data_ptr(),
                h_items=items.ctypes.data, num_items=len(items),
                d_scratch=scratch.data_ptr() if use_scratch else None,
                d_item_times=None, d_bin_offsets=None, waves_per_simd=0)
    stream = torch.cuda.current_stream()
    st = fn(ctypes.byref(batch.c_batch), ctypes.byref(s), surv.data_ptr(), cap, counts.data_ptr(),
            total.data_ptr(), None, ctypes.c_void_p(stream.cuda_stream))
    L.check("enumerate", st)
    torch.cuda.synchronize()
    tot = total.cpu().numpy()
    rec = surv[:int(tot[1])].cpu().numpy()
    rec = rec[rec[:, 1] != -1]
    rec = rec[np.lexsort((rec[:, 0], rec[:, 1]))]
    return counts.cpu().numpy(), tot, rec


def test_noalloc_matches_enumerate_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import _lib as L, engine as E
    lib = L.lib()
    big = E.prepare_many([i for i in W.batch(E.kdim, count=64) if i.meta["k"] <= 20][:24])
    small = big[:5]
    for name, preps in (("first call", big), ("second call, smaller batch", small)):
        batch = E.DeviceBatch(preps)
        items = E.build_queue(batch.k, 9, 128, cost=np.ones(len(preps), np.float32), order=1)
        _say(f"[no-alloc] {name}: {len(preps)} instances, {len(items)} items")
        want = _run(E, L, batch, items, lib.wpm_enumerate, True)
        got = _run(E, L, batch, items, lib.wpm_enumerate_noalloc, False)
        assert np.array_equal(got[0], want[0]), name
        assert np.array_equal(got[1][[0, 2, 3]], want[1][[0, 2, 3]]) and got[1][2] == 0, name
        assert np.array_equal(got[2], want[2]), name
        assert int(want[0].sum()) == len(want[2]) > 0


def test_noalloc_rejects_a_workspace_argument():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_00806_amd import _lib as L, engine as E
    preps = E.prepare_many([i for i in W.batch(E.kdim, count=8)][:2])
    batch = E.DeviceBatch(preps)
    scratch = torch.zeros(4, dtype=torch.int64, device="cuda")
    s = L.Sched(mode=L.SCHED_DYNAMIC, wg_size=128, num_items=0, d_scratch=scratch.data_ptr())
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    st = L.lib().wpm_enumerate_noalloc(ctypes.byref(batch.c_batch), ctypes.byref(s), out.data_ptr(), 1,
                                        out.data_ptr(), out.data_ptr(), None, None)
    assert st == L.WPM_EINVAL
