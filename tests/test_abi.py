"""The C ABI library loads and exports every function include/*.h declares
(no GPU: only loading, symbol lookup and host-only entry points)."""
import ctypes
import glob
import os
import re

import pytest

from conftest import ROOT


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def fdlib():
    import paper_2609_15034_amd as fd
    if not os.path.exists(fd.LIB_PATH):
        import paper_2609_15034_amd.build as b
        b.build()
    return fd


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("fsst_decode", "onpair_decode", "fd_decode", "fd_dict_create", "fd_workspace_size"):
        assert n in names


def test_library_exports_every_declared_function(fdlib):
    L = ctypes.CDLL(fdlib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_entry_points(fdlib):
    fd = fdlib
    assert fd.status_str(0) == "FD_OK" and fd.status_str(7) == "FD_EOFFSETS" and fd.status_str(99) == "FD_UNKNOWN"
    assert "gfx950" in fd.version()
    assert fd.decoded_bound("fsst8", 10) == 80 and fd.decoded_bound("onpair16", 10) == 160
    a = fd.workspace_size("fsst8", 1000, 10)
    b = fd.workspace_size("fsst8", 1000, 10, {"mode": 0, "tile_codes": 16, "grid": 0, "reserved": 0})
    assert b >= a > 0
    # OnPair one-shot decodes repack the dictionary inside the workspace
    assert fd.workspace_size("onpair16", 1000, 10) > 65536 * 17
    with pytest.raises(fd.DecodeError):
        fd.workspace_size("fsst8", -1, 10)
    # tile sizes: whole 16-byte chunks of codes, at most one pass less a chunk
    for codec, bad in (("fsst8", 8), ("fsst8", 24), ("fsst8", 8192), ("onpair16", 4), ("onpair16", 4096),
                       ("onpair12", 12), ("fsst8", -16)):
        with pytest.raises(fd.DecodeError):
            fd.workspace_size(codec, 10, 10, {"mode": 0, "tile_codes": bad, "grid": 0, "reserved": 0})
    for codec, good in (("fsst8", 16), ("fsst8", 8176), ("onpair16", 8), ("onpair12", 4088)):
        assert fd.workspace_size(codec, 10, 10, {"mode": 0, "tile_codes": good, "grid": 0, "reserved": 0}) > 0


def test_argument_errors_enqueue_nothing(fdlib):
    """Host-side checks reject bad arguments before touching the device."""
    L = fdlib.lib()
    P = ctypes.c_void_p
    fake = P(1 << 20)   # never dereferenced: the call must fail before any launch
    ws = P(1 << 21)
    # index_bits 16
    st = L.fsst_decode(fake, 10, fake, 16, 1, fake, fake, 1, fake, fake, 10, ws, 1 << 20, None, 0, None)
    assert st == fdlib.EINVAL
    # workspace too small
    st = L.fsst_decode(fake, 10, fake, 64, 1, fake, fake, 1, fake, fake, 10, ws, 8, None, 0, None)
    assert st == fdlib.EINVAL
    # async without a status pointer
    st = L.fsst_decode(fake, 10, fake, 64, 1, fake, fake, 1, fake, fake, 10, ws, 1 << 20, None, 1, None)
    assert st == fdlib.EINVAL
    # too many symbols / tokens
    st = L.fsst_decode(fake, 10, fake, 64, 1, fake, fake, 256, fake, fake, 10, ws, 1 << 20, None, 0, None)
    assert st == fdlib.EINVAL
    st = L.onpair_decode(fake, 10, fake, 64, 1, fake, fake, 65537, fake, fake, 10, ws, 1 << 22, None, 0, None)
    assert st == fdlib.EINVAL
    # odd address for uint16 codes
    st = L.onpair_decode(P((1 << 20) + 1), 10, fake, 64, 1, fake, fake, 1, fake, fake, 10, ws, 1 << 22, None, 0, None)
    assert st == fdlib.EINVAL
    # negative sizes, null workspace
    st = L.fsst_decode(fake, -1, fake, 64, 1, fake, fake, 1, fake, fake, 10, ws, 1 << 20, None, 0, None)
    assert st == fdlib.EINVAL
    st = L.fsst_decode(fake, 10, fake, 64, 1, fake, fake, 1, fake, fake, 10, None, 1 << 20, None, 0, None)
    assert st == fdlib.EINVAL
    # misaligned workspace
    st = L.fsst_decode(fake, 10, fake, 64, 1, fake, fake, 1, fake, fake, 10, P((1 << 21) + 8), 1 << 20, None, 0,
                       None)
    assert st == fdlib.EINVAL
    # null dictionary handle
    assert L.fd_decode(None, fake, 10, fake, 64, 1, fake, fake, 10, ws, 1 << 20, None, 0, None) == fdlib.EINVAL


def test_batch_argument_errors_enqueue_nothing(fdlib):
    """batch_decode rejects bad batches on the host, before touching the device."""
    L = fdlib.lib()
    P = ctypes.c_void_p
    ws = P(1 << 21)
    arr = (fdlib.Column * 1)()
    assert L.batch_decode(arr, -1, None, ws, 1 << 20, None, 0, None) == fdlib.EINVAL          # n_cols < 0
    assert L.batch_decode(None, 1, None, ws, 1 << 20, None, 0, None) == fdlib.EINVAL          # no column array
    assert L.batch_decode(arr, 0, None, None, 1 << 20, None, 0, None) == fdlib.EINVAL        # no workspace
    assert L.batch_decode(arr, 0, None, P((1 << 21) + 8), 1 << 20, None, 0, None) == fdlib.EINVAL   # misaligned
    assert L.batch_decode(arr, 0, None, ws, 1 << 20, None, 1, None) == fdlib.EINVAL          # async, no status
    assert L.batch_decode(arr, 0, None, ws, 1 << 20, None, 8, None) == fdlib.EINVAL          # unknown flag
    tu = fdlib.Tuning(2, 0, 0, 0)                                                             # no such mode
    assert L.batch_decode(arr, 0, ctypes.byref(tu), ws, 1 << 20, None, 0, None) == fdlib.EINVAL
    arr[0] = fdlib.Column(0, 1 << 20, 10, 1 << 20, 64, 1, 1 << 20, 1 << 20, 10)               # no dictionary
    assert L.batch_decode(arr, 1, None, ws, 1 << 20, None, 0, None) == fdlib.EINVAL
    sz = ctypes.c_size_t(0)
    assert L.fd_batch_workspace_size(arr, 1, None, ctypes.byref(sz)) == fdlib.EINVAL
    assert L.fd_batch_workspace_size(arr, 0, None, ctypes.byref(sz)) == 0 and sz.value >= 256
    assert L.fd_batch_workspace_size(arr, -1, None, ctypes.byref(sz)) == fdlib.EINVAL


def test_sidecar_host_checks(fdlib):
    """fd_sidecar_layout follows the tiling; the sidecar entry points reject a
    missing dictionary, a sidecar of another tiling and three-phase tuning
    before touching the device."""
    fd = fdlib
    tu = {"mode": 0, "tile_codes": 48, "grid": 0, "reserved": 0}
    assert fd.sidecar_layout("fsst8", 1000, 10, tu) == (48, 22)        # ceil(1000 / 48) + 1
    assert fd.sidecar_layout("onpair12", 0, 0, tu) == (48, 2)          # one tile even without codes
    T, n = fd.sidecar_layout("onpair16", 10 ** 6, 10 ** 4)
    assert T == 4088 and n == -(-10 ** 6 // T) + 1
    assert fd.sidecar_layout("fsst8", 10 ** 6, 10 ** 4) == (8176, -(-10 ** 6 // 8176) + 1)
    with pytest.raises(fd.DecodeError):
        fd.sidecar_layout("fsst8", 1000, 10, {"mode": 1, "tile_codes": 0, "grid": 0, "reserved": 0})
    L = fd.lib()
    P = ctypes.c_void_p
    fake, ws = P(1 << 20), P(1 << 21)
    assert L.fd_sidecar_build(None, fake, 10, fake, 64, 1, fake, 2, ws, 1 << 20, None, 0, None, None) == fd.EINVAL
    assert L.fd_decode_sidecar(None, fake, 10, fake, 64, 1, fake, 2, fake, fake, 10, ws, 1 << 20, None, 0, None,
                               None) == fd.EINVAL
    assert fd.status_str(fd.ESIDECAR) == "FD_ESIDECAR"


def test_take_host_checks(fdlib):
    """fd_take_workspace_size grows with the code budget and plans one
    workspace for both modes (an unknown mode is rejected); fd_decode_take
    rejects a missing dictionary."""
    fd = fdlib
    a = fd.take_workspace_size("fsst8", 10 ** 6, 10 ** 4, 100, 0)
    b = fd.take_workspace_size("fsst8", 10 ** 6, 10 ** 4, 100, 10 ** 5)
    c = fd.take_workspace_size("onpair12", 10 ** 6, 10 ** 4, 100, 10 ** 5)
    assert b - a >= 10 ** 5 - 256 and c - b >= 10 ** 5 - 256    # 256-byte rounding; OnPair-12 codes widen to 16 bits
    assert fd.take_workspace_size("onpair16", 0, 0, 0, 0) > 0
    for bad in ((10 ** 6, 10 ** 4, -1, 0), (10 ** 6, 10 ** 4, 1, -1)):
        with pytest.raises(fd.DecodeError):
            fd.take_workspace_size("fsst8", *bad)
    # both modes plan the same workspace; there is no third mode
    assert fd.take_workspace_size("fsst8", 100, 10, 5, 100, {"mode": 1, "tile_codes": 0, "grid": 0, "reserved": 0}) == \
        fd.take_workspace_size("fsst8", 100, 10, 5, 100, {"mode": 0, "tile_codes": 0, "grid": 0, "reserved": 0})
    with pytest.raises(fd.DecodeError):
        fd.take_workspace_size("fsst8", 100, 10, 5, 100, {"mode": 2, "tile_codes": 0, "grid": 0, "reserved": 0})
    L = fd.lib()
    P = ctypes.c_void_p
    fake, ws = P(1 << 20), P(1 << 21)
    assert L.fd_decode_take(None, fake, 10, fake, 64, 1, fake, 1, 10, fake, fake, 10, ws, 1 << 20, None, 0, None,
                            None) == fd.EINVAL


def test_profile_host_checks(fdlib):
    """fd_profile_begin rejects an empty or unknown kind mask and bad pool
    sizes; fd_profile_end with no open profile is an error (no device calls)."""
    L = fdlib.lib()
    assert L.fd_profile_begin(0, 16) == fdlib.EINVAL
    assert L.fd_profile_begin(1 << 6, 16) == fdlib.EINVAL
    assert L.fd_profile_begin(1, 0) == fdlib.EINVAL
    assert L.fd_profile_begin(1, (1 << 20) + 1) == fdlib.EINVAL
    assert L.fd_profile_end(None, None, None, None, None) == fdlib.EINVAL
    assert fdlib.PROF_KINDS[4] == "decode" and len(fdlib.PROF_KINDS) == 6


def test_server_status_names(fdlib):
    fd = fdlib
    assert [fd.status_str(k) for k in (fd.ETIMEOUT, fd.ECANCELED, fd.EBUSY)] == ["FD_ETIMEOUT", "FD_ECANCELED",
                                                                              "FD_EBUSY"]
    L = fd.lib()
    assert L.fd_server_cancel(None, 1) == fd.EINVAL
    assert L.fd_server_wait_for(None, 1, 0, None, None) == fd.EINVAL
