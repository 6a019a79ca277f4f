"""The batch autotuner (fd_batch_autotune): the residency model prunes the
candidates of a batch that fills the device, small batches try the smaller
tiles, choices are cached per shape in the process and, with
FD_AUTOTUNE_CACHE set, in a file read back later; batches decoded with the
chosen tuning equal the oracle."""
import os

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


def columns(srcs):
    import torch
    import paper_2609_15034_amd as fd
    tups = []
    for c in srcs:
        codes_np = c.codes.view(np.int16) if c.codec == "onpair16" else c.codes
        d = fd.Dict(c.codec, torch.from_numpy(c.dict_bytes).cuda(), torch.from_numpy(c.dict_lens).cuda())
        off = torch.from_numpy(c.code_off).cuda()
        tups.append((d, torch.from_numpy(codes_np.copy()).cuda(), off,
                     torch.full((c.n_strings + 1,), -7, dtype=off.dtype, device="cuda"),
                     torch.full((c.decoded_bytes + 64,), 0xA5, dtype=torch.uint8, device="cuda")))
    return tups


def check(srcs, tups):
    for c, t in zip(srcs, tups):
        assert np.array_equal(t[3].cpu().numpy().astype(np.int64), c.text_off)
        out = t[4].cpu().numpy()
        assert np.array_equal(out[:c.decoded_bytes], c.text) and np.all(out[c.decoded_bytes:] == 0xA5)


def test_small_batch_tries_smaller_tiles_and_caches(datagen_mod, tmp_path):
    import torch
    import paper_2609_15034_amd as fd
    srcs = [datagen_mod.fsst_small(seed=91, n_strings=500), datagen_mod.fsst_small(seed=92, n_strings=700),
            datagen_mod.onpair_urls(seed=93, target_bytes=64 << 10, sample_bytes=64 << 10)]
    tups = columns(srcs)
    ws = torch.empty(fd.batch_workspace_size(tups, None), dtype=torch.uint8, device="cuda")
    cache = tmp_path / "tune.txt"
    os.environ["FD_AUTOTUNE_CACHE"] = str(cache)
    try:
        fd.debug_autotune_forget()
        c0 = fd.batch_autotune(tups, ws)
        assert c0["source"] == 0 and c0["candidates_timed"] >= 4      # both modes, several tile sizes
        assert c0["mode"] in (0, 1) and c0["tile_scale_pct"] in (100, 50, 25) and c0["grid_pct"] in (100, 75)
        c1 = fd.batch_autotune(tups, ws)
        assert c1["source"] == 1 and c1["candidates_timed"] == 0
        assert {k: c1[k] for k in ("mode", "tile_scale_pct", "grid_pct")} == \
               {k: c0[k] for k in ("mode", "tile_scale_pct", "grid_pct")}
        lines = cache.read_text().split("\n")
        assert lines[0].startswith("fastdecode-autotune 1 ") and len([x for x in lines if x]) == 1
        fd.debug_autotune_forget()
        c2 = fd.batch_autotune(tups, ws)
        assert c2["source"] == 2
        assert {k: c2[k] for k in ("mode", "tile_scale_pct", "grid_pct")} == \
               {k: c0[k] for k in ("mode", "tile_scale_pct", "grid_pct")}
    finally:
        del os.environ["FD_AUTOTUNE_CACHE"]
        fd.debug_autotune_forget()
    for t in tups:
        t[3].fill_(-7)
        t[4].fill_(0xA5)
    status = torch.full((len(tups) + 1,), -1, dtype=torch.int32, device="cuda")
    assert fd.batch_decode(tups, ws, status=status, async_=True) == fd.OK
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * (len(tups) + 1)
    check(srcs, tups)


def test_large_batch_is_pruned(datagen_mod):
    """One 64 MiB column fills the device many times over with the largest
    tiles: only those are timed (mode 0 at both workgroup counts, mode 1)."""
    import torch
    import paper_2609_15034_amd as fd
    srcs = [datagen_mod.fsst_logs(seed=94, target_bytes=64 << 20)]
    tups = columns(srcs)
    ws = torch.empty(fd.batch_workspace_size(tups, None), dtype=torch.uint8, device="cuda")
    fd.debug_autotune_forget()
    c = fd.batch_autotune(tups, ws)
    assert c["source"] == 0 and c["candidates_timed"] == 3 and c["tile_scale_pct"] == 100
    check(srcs, tups)          # the timed runs decoded the batch
    fd.debug_autotune_forget()
