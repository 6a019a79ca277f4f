"""CPU ORACLE (pure-Python transcription) - test infrastructure only.

A direct, tiny restatement of the decode semantics for brute force over tiny
inputs (background section on dictionary-compressed strings): each code looks
up a token and the tokens are concatenated in code order; for FSST-8 the
reserved escape code (255) is followed by one literal byte.  Returns
``(status, out_off, out)`` with the status numbering of ``oracle``.
"""
from __future__ import annotations

OK, EINVAL, EBADCODE, EESCAPE, ECAPACITY, EOVERFLOW, EBADDICT, EOFFSETS = range(8)
ESCAPE = 255


def decode_fsst8(codes: bytes, code_off: list[int], syms: list[bytes]):
    if any(len(s) == 0 or len(s) > 8 for s in syms) or len(syms) > 255:
        return EBADDICT, None, None
    if code_off[0] < 0 or code_off[-1] > len(codes) or any(b < a for a, b in zip(code_off, code_off[1:])):
        return EOFFSETS, None, None
    out = bytearray()
    out_off = [0]
    for i in range(len(code_off) - 1):
        p, e = code_off[i], code_off[i + 1]
        while p < e:
            c = codes[p]
            if c == ESCAPE:
                if p + 1 >= e:
                    return EESCAPE, None, None
                out.append(codes[p + 1])
                p += 2
            else:
                if c >= len(syms):
                    return EBADCODE, None, None
                out += syms[c]
                p += 1
        out_off.append(len(out))
    return OK, out_off, bytes(out)


def decode_onpair16(codes: list[int], code_off: list[int], toks: list[bytes]):
    if any(len(t) == 0 or len(t) > 16 for t in toks) or len(toks) > 65536:
        return EBADDICT, None, None
    if code_off[0] < 0 or code_off[-1] > len(codes) or any(b < a for a, b in zip(code_off, code_off[1:])):
        return EOFFSETS, None, None
    out = bytearray()
    out_off = [0]
    for i in range(len(code_off) - 1):
        for p in range(code_off[i], code_off[i + 1]):
            c = codes[p]
            if c >= len(toks):
                return EBADCODE, None, None
            out += toks[c]
        out_off.append(len(out))
    return OK, out_off, bytes(out)
