"""Served decode (fd_server): requests decoded in the mix of continuous
batching are byte-identical to the same requests decoded alone, admission
keeps the device bytes in flight within the budget, and every request's
status is its own."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_15034_amd as fd
    fd.lib()
    yield


@pytest.fixture(scope="module")
def pool(datagen_mod):
    return datagen_mod.serve_pool(seed=51, n_dicts=6, n_chunks=10, min_bytes=16 << 10, max_bytes=2 << 20)


class Req:
    def __init__(self, chunk, d):
        import torch
        self.chunk = chunk
        self.d = d
        self.codes = torch.from_numpy(chunk.codes.copy()).cuda()
        if chunk.codec == "onpair16":
            self.codes = self.codes.view(torch.int16)
        self.code_off = torch.from_numpy(chunk.code_off.copy()).cuda()
        self.out = torch.full((chunk.decoded_bytes + 64,), 0xA5, dtype=torch.uint8, device="cuda")
        self.off = torch.full((chunk.n_strings + 1,), -7, dtype=self.code_off.dtype, device="cuda")

    def tup(self):
        return (self.d, self.codes, self.code_off, self.off, self.out)


def make_dicts(pool):
    import torch
    import paper_2609_15034_amd as fd
    out = []
    for codec, db, dl in pool.dicts:
        out.append(fd.Dict(codec, torch.from_numpy(db).cuda(), torch.from_numpy(dl).cuda()))
    return out


def alone(r):
    import torch
    import paper_2609_15034_amd as fd
    ws = fd.alloc_workspace(r.d.codec, r.codes.numel(), r.code_off.numel() - 1)
    out = torch.full_like(r.out, 0xA5)
    off = torch.empty_like(r.off)
    st = fd.decode_into(r.d, r.codes, r.code_off, off, out, ws)
    return st, off.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("budget,slots,max_batch", [(0, 4, 64), (6 << 20, 3, 2), (1, 2, 1)])
def test_served_equals_alone(pool, budget, slots, max_batch):
    import torch
    import paper_2609_15034_amd as fd
    dicts = make_dicts(pool)
    reqs = [Req(c, dicts[k]) for c, k in zip(pool.chunks, pool.chunk_dict)] * 1
    reqs += [Req(c, dicts[k]) for c, k in zip(pool.chunks[::-1], pool.chunk_dict[::-1])]
    ref = [alone(r) for r in reqs]
    torch.cuda.synchronize()
    recs = [fd.Server.prepare(r.tup()) for r in reqs[::2]]     # every other request as a prepared record
    with fd.Server(max_inflight_bytes=budget, n_slots=slots, max_batch=max_batch) as srv:
        tickets = [srv.submit(recs[k // 2] if k % 2 == 0 else r.tup()) for k, r in enumerate(reqs)]
        res = [srv.wait(t) for t in tickets]
        stats = srv.stats()
    for r, (st, lat), (st0, off0, out0) in zip(reqs, res, ref):
        assert st == 0 and st0 == 0
        assert lat > 0
        assert np.array_equal(r.off.cpu().numpy(), off0)
        assert np.array_equal(r.out.cpu().numpy(), out0)       # bytes and the untouched tail
        assert np.array_equal(out0[:r.chunk.decoded_bytes], r.chunk.text)
    assert stats["submitted"] == stats["admitted"] == stats["completed"] == len(reqs)
    if budget > 1:
        assert stats["max_inflight_bytes"] <= budget
    if max_batch == 1:
        assert stats["batches"] == len(reqs)


def test_served_against_oracle_and_errors(pool):
    """Served results equal the oracle's; a request whose dictionary lacks some
    of its codes fails with the oracle's status while the others succeed."""
    import torch
    import oracle
    import paper_2609_15034_amd as fd
    dicts = make_dicts(pool)
    reqs = [Req(c, dicts[k]) for c, k in zip(pool.chunks[:4], pool.chunk_dict[:4])]
    fi = next(i for i, k in enumerate(pool.chunk_dict) if pool.dicts[k][0] == "fsst8")
    chunk = pool.chunks[fi]
    _, db, dl = pool.dicts[pool.chunk_dict[fi]]
    keep = 200
    db2, dl2 = db[:int(dl[:keep].sum())], dl[:keep]
    d2 = fd.Dict("fsst8", torch.from_numpy(db2.copy()).cuda(), torch.from_numpy(dl2.copy()).cuda())
    bad = Req(chunk, d2)
    exp_bad = oracle.decode("fsst8", chunk.codes, chunk.code_off, db2, dl2, out_capacity=bad.out.numel())
    assert exp_bad.status != 0
    with fd.Server(n_slots=2, max_batch=3) as srv:
        tickets = [srv.submit(r.tup()) for r in reqs + [bad]]
        res = [srv.wait(t) for t in tickets]
    for r, (st, _) in zip(reqs, res[:-1]):
        c = r.chunk
        exp = oracle.decode(c.codec, c.codes, c.code_off, c.dict_bytes, c.dict_lens, out_capacity=r.out.numel())
        assert st == exp.status == 0
        assert np.array_equal(r.off.cpu().numpy(), exp.out_off)
        assert np.array_equal(r.out.cpu().numpy()[:len(exp.out_bytes)], exp.out_bytes)
    assert res[-1][0] == exp_bad.status


def test_server_rejects_bad_requests(pool):
    """A request with a host-visible error is refused at submission."""
    import ctypes
    import paper_2609_15034_amd as fd
    dicts = make_dicts(pool)
    r = Req(pool.chunks[0], dicts[pool.chunk_dict[0]])
    L = fd.lib()
    with fd.Server() as srv:
        arr = fd.make_columns([r.tup()])
        arr[0].index_bits = 48
        t = ctypes.c_uint64(0)
        assert L.fd_server_submit(srv._h, arr, ctypes.byref(t)) == fd.EINVAL
        arr = fd.make_columns([r.tup()])
        arr[0].dict = None
        assert L.fd_server_submit(srv._h, arr, ctypes.byref(t)) == fd.EINVAL
        ticket = srv.submit(r.tup())
        assert srv.wait(ticket)[0] == 0


def check_untouched(r):
    """A request that never ran: its outputs hold their canary values."""
    assert np.all(r.out.cpu().numpy() == 0xA5)
    assert np.all(r.off.cpu().numpy() == -7)


def check_decoded(r, st):
    assert st == 0
    c = r.chunk
    assert np.array_equal(r.out.cpu().numpy()[:c.decoded_bytes], c.text)
    assert np.array_equal(r.off.cpu().numpy().astype(np.int64), c.text_off)


def test_wait_with_timeout_and_cancel(pool):
    """One slot, one request per batch: a request queued behind many is not
    done after a 1 us wait (FD_ETIMEOUT, the ticket stays valid), and queued
    requests can be cancelled (FD_ECANCELED, outputs untouched); the others
    decode exactly."""
    import paper_2609_15034_amd as fd
    dicts = make_dicts(pool)
    big = max(range(len(pool.chunks)), key=lambda i: pool.chunks[i].decoded_bytes)
    reqs = [Req(pool.chunks[big], dicts[pool.chunk_dict[big]]) for _ in range(24)]
    with fd.Server(n_slots=1, max_batch=1) as srv:
        tickets = [srv.submit(r.tup()) for r in reqs]
        assert srv.wait(tickets[-1], timeout_us=1) is None        # 23 requests ahead of it
        cancelled = [srv.cancel(t) for t in tickets[-6:]]
        res = [srv.wait(t) for t in tickets]
        with pytest.raises(fd.DecodeError):
            srv.wait(tickets[0])                                  # each ticket is waited for once
        with pytest.raises(fd.DecodeError):
            srv.cancel(tickets[0])
        stats = srv.stats()
    assert cancelled[-1]                                          # the last one was still queued
    n_cancelled = 0
    for r, (st, lat), was in zip(reqs, res, [False] * 18 + cancelled):
        if was:
            assert st == fd.ECANCELED
            check_untouched(r)
            n_cancelled += 1
        else:
            check_decoded(r, st)
    assert stats["canceled"] == n_cancelled and stats["completed"] == len(reqs)
    assert stats["admitted"] == len(reqs) - n_cancelled


def test_queue_deadline(pool):
    """With a 1 us queue deadline and one slot, requests that wait for
    admission complete with FD_ETIMEOUT without running; the admitted ones
    decode exactly."""
    import paper_2609_15034_amd as fd
    dicts = make_dicts(pool)
    big = max(range(len(pool.chunks)), key=lambda i: pool.chunks[i].decoded_bytes)
    reqs = [Req(pool.chunks[big], dicts[pool.chunk_dict[big]]) for _ in range(16)]
    with fd.Server(n_slots=1, max_batch=1, queue_timeout_us=1) as srv:
        tickets = [srv.submit(r.tup()) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        stats = srv.stats()
    n_timed_out = 0
    for r, (st, _) in zip(reqs, res):
        if st == fd.ETIMEOUT:
            check_untouched(r)
            n_timed_out += 1
        else:
            check_decoded(r, st)
    assert n_timed_out >= 1 and stats["timed_out"] == n_timed_out
    assert stats["admitted"] + n_timed_out == len(reqs)
