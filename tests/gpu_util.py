"""Helpers for GPU parity tests: run the HIP decoder through the C ABI on
seeded columns and compare with the CPU oracle element by element."""
from __future__ import annotations

import numpy as np

GUARD = 64
CANARY = 0xA5


def torch_mod():
    import torch
    return torch


def to_dev(a: np.ndarray, misalign: int = 0):
    """Copy a numpy array to the GPU; with misalign > 0 the returned tensor
    starts `misalign` bytes into a larger buffer (an unaligned pointer)."""
    torch = torch_mod()
    a = np.ascontiguousarray(a)
    if misalign:
        raw = np.frombuffer(a.tobytes(), np.uint8)
        buf = torch.zeros(len(raw) + misalign + 16, dtype=torch.uint8, device="cuda")
        buf[misalign:misalign + len(raw)] = torch.from_numpy(raw.copy()).cuda()
        return buf, buf[misalign:misalign + len(raw)]
    t = torch.from_numpy(a.copy()).cuda()
    return t, t


class GuardedOut:
    """out_bytes / out_offsets with canary guard bands on both sides."""

    def __init__(self, cap: int, n_off: int, idx_dtype, out_misalign: int = 0):
        torch = torch_mod()
        self.cap = cap
        self.pad = GUARD + out_misalign
        self.buf = torch.full((self.pad + cap + GUARD,), CANARY, dtype=torch.uint8, device="cuda")
        self.out = self.buf[self.pad:self.pad + cap]
        self.obuf = torch.full((n_off + 2 * 16,), -7, dtype=idx_dtype, device="cuda")
        self.off = self.obuf[16:16 + n_off]

    def check_guards(self):
        b = self.buf.cpu().numpy()
        assert np.all(b[:self.pad] == CANARY), "write before out_bytes"
        assert np.all(b[self.pad + self.cap:] == CANARY), "write past out_capacity"
        o = self.obuf.cpu().numpy()
        assert np.all(o[:16] == -7) and np.all(o[-16:] == -7), "write outside out_offsets"


def gpu_decode(col_codec, codes, code_off, dict_bytes, dict_lens, *, via="dict", tuning=None, cap=None,
               codes_misalign=0, out_misalign=0, async_=False, code_slice=None):
    """Decode on the GPU.  Returns (status, out_off np.int64, out_bytes np.uint8, guards)."""
    import paper_2609_15034_amd as fd
    torch = torch_mod()
    _, codes_t = to_dev(codes, codes_misalign)
    if col_codec == "onpair16" and codes_misalign:
        codes_t = codes_t.view(torch.int16)
    elif col_codec == "onpair16":
        codes_t = codes_t.view(torch.int16)
    off_t = torch.from_numpy(np.ascontiguousarray(code_off)).cuda()
    db = torch.from_numpy(np.ascontiguousarray(dict_bytes, np.uint8)).cuda() if len(dict_bytes) else \
        torch.zeros(1, dtype=torch.uint8, device="cuda")
    dl = torch.from_numpy(np.ascontiguousarray(dict_lens, np.uint8)).cuda()
    n_codes = len(codes)
    n_strings = len(code_off) - 1
    maxlen = 8 if col_codec == "fsst8" else 16
    if cap is None:
        cap = n_codes * maxlen
    g = GuardedOut(cap, n_strings + 1, off_t.dtype, out_misalign)
    ws = fd.alloc_workspace(col_codec, n_codes, n_strings, tuning)
    status_t = torch.full((1,), -1, dtype=torch.int32, device="cuda") if async_ else None
    if via == "dict":
        d = fd.Dict(col_codec, db[:len(dict_bytes)] if len(dict_bytes) else db, dl)
        st = fd.decode_into(d, codes_t, off_t, g.off, g.out, ws, status=status_t, async_=async_, tuning=tuning,
                            n_codes=n_codes)
    elif col_codec == "fsst8":
        st = fd.fsst_decode(codes_t, off_t, db, dl, g.off, g.out, ws, status=status_t, async_=async_)
    else:
        st = fd.onpair_decode(codes_t, off_t, db, dl, g.off, g.out, ws, status=status_t, async_=async_)
    if async_:
        assert st == fd.OK
        torch.cuda.synchronize()
        st = int(status_t.item())
    torch.cuda.synchronize()
    g.check_guards()
    return st, g.off.cpu().numpy().astype(np.int64), g.out.cpu().numpy(), g


def assert_parity(col_codec, codes, code_off, dict_bytes, dict_lens, **kw):
    """GPU vs oracle: status, offsets and bytes must be identical."""
    import oracle
    exp = oracle.decode(col_codec, codes, code_off, dict_bytes, dict_lens, out_capacity=kw.get("cap"))
    st, off, out, _ = gpu_decode(col_codec, codes, code_off, dict_bytes, dict_lens, **kw)
    assert st == exp.status, (st, exp.status)
    if exp.status in (0, 4):   # offsets complete on OK and ECAPACITY
        if not np.array_equal(off, exp.out_off):
            bad = np.nonzero(off != exp.out_off)[0]
            raise AssertionError(f"offsets differ at {bad[:10]} (of {len(bad)}): gpu {off[bad[:5]]} "
                                 f"oracle {exp.out_off[bad[:5]]}")
        n = len(exp.out_bytes)
        if not np.array_equal(out[:n], exp.out_bytes):
            bad = np.nonzero(out[:n] != exp.out_bytes)[0]
            raise AssertionError(f"bytes differ at {bad[:10]} (of {len(bad)})")
    return exp
