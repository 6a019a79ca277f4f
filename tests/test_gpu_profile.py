"""The library's kernel timing (fd_profile_begin / fd_profile_end): every
launch of a selected kind is timed on its own stream, the others are not,
launches past the event pool are counted as dropped, and timing changes no
output."""
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


def test_profile_counts_and_output(datagen_mod):
    import torch
    import oracle
    import paper_2609_15034_amd as fd
    c = datagen_mod.fsst_logs(target_bytes=4 << 20)
    codes = torch.from_numpy(c.codes).cuda()
    off = torch.from_numpy(c.code_off).cuda()
    d = fd.Dict("fsst8", torch.from_numpy(c.dict_bytes).cuda(), torch.from_numpy(c.dict_lens).cuda())
    exp = oracle.decode("fsst8", c.codes, c.code_off, c.dict_bytes, c.dict_lens)
    s = torch.cuda.Stream()
    for mode in (0, 1):
        tu = {"mode": mode, "tile_codes": 0, "grid": 0, "reserved": 0}
        ws = fd.alloc_workspace("fsst8", len(c.codes), c.n_strings, tu)
        out = torch.zeros(c.decoded_bytes, dtype=torch.uint8, device="cuda")
        oo = torch.zeros(c.n_strings + 1, dtype=off.dtype, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        fd.profile_begin(("decode", "totals"), 3)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):                  # launches on a side stream are timed on it
            for _ in range(4):
                assert fd.decode_into(d, codes, off, oo, out, ws, status=status, async_=True, tuning=tu,
                                      stream=s) == fd.OK
        s.synchronize()
        p = fd.profile_end()
        assert int(status.item()) == 0
        assert np.array_equal(out.cpu().numpy(), exp.out_bytes)
        assert np.array_equal(oo.cpu().numpy().astype(np.int64), exp.out_off)
        assert "reset" not in p and "coarse" not in p and "scan" not in p
        if mode == 0:
            assert p["decode"]["launches"] == 3 and p["dropped"] == 1 and "totals" not in p
        else:
            assert p["decode"]["launches"] + p["totals"]["launches"] == 3 and p["dropped"] == 5
        for k in ("decode", "totals"):
            if k in p:
                assert 0 < p[k]["min_us"] <= p[k]["mean_us"] <= p[k]["max_us"] < 1e6
    with pytest.raises(fd.DecodeError):
        fd.profile_end()                            # nothing open
    fd.profile_begin(("reset",), 1)
    with pytest.raises(fd.DecodeError):
        fd.profile_begin(("reset",), 1)             # one at a time
    assert fd.profile_end()["dropped"] == 0
