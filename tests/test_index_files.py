"""Index files without a GPU: loading a missing, foreign, truncated,
inconsistent or altered file fails with BBC_EINVAL before any device work."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


def _header(quant=0, metric=0, storage=0, d=8, nlist=2, pq_m=2, pq_bits=8, n=4, eps0=0.0):
    h = np.zeros(56, np.uint8)
    h[:8] = np.frombuffer(b"BBCIDX2\0", np.uint8)
    h[8:40] = np.array([quant, metric, storage, d, nlist, pq_m, pq_bits, 0], np.int32).view(np.uint8)
    h[40:48] = np.array([n], np.int64).view(np.uint8)
    h[48:52] = np.array([eps0], np.float32).view(np.uint8)
    return h


def _load_rc(bbc, path):
    import ctypes as C
    h = C.c_void_p()
    return bbc.load().bbc_index_load(0, str(path).encode(), C.byref(h)), h.value


def test_missing_and_foreign_files(bbc, tmp_path):
    rc, h = _load_rc(bbc, tmp_path / "none.bbc")
    assert rc == bbc.EINVAL and h is None
    p = tmp_path / "foreign.bbc"
    p.write_bytes(b"not an index file at all, just text" * 4)
    assert _load_rc(bbc, p)[0] == bbc.EINVAL
    assert "not an index file" in bbc.load().bbc_last_error().decode()


@pytest.mark.parametrize("fields", [dict(quant=3), dict(d=1028), dict(d=6), dict(nlist=0), dict(n=0),
                                    dict(pq_bits=6), dict(pq_m=3), dict(quant=1, d=96), dict(storage=2)])
def test_header_out_of_range(bbc, tmp_path, fields):
    p = tmp_path / "bad.bbc"
    _header(**fields).tofile(p)
    assert _load_rc(bbc, p)[0] == bbc.EINVAL


def test_size_must_match_the_header(bbc, tmp_path):
    # PQ, n = 4, d = 8, nlist = 2, 2 x 8-bit: 56 + 64 + 24 + 32 + 256*4*2*... bytes
    n, d, nlist, m, bits = 4, 8, 2, 2, 8
    body = 4 * nlist * d + 8 * (nlist + 1) + 8 * n + 4 * m * (1 << bits) * (d // m) + n * m + 4 * n * d
    p = tmp_path / "short.bbc"
    np.concatenate([_header(), np.zeros(body - 1, np.uint8)]).tofile(p)
    assert _load_rc(bbc, p)[0] == bbc.EINVAL
    assert "size" in bbc.load().bbc_last_error().decode()
    np.concatenate([_header(), np.zeros(body + 16, np.uint8)]).tofile(p)
    assert _load_rc(bbc, p)[0] == bbc.EINVAL
    # the arrays without their checksum
    np.concatenate([_header(), np.zeros(body, np.uint8)]).tofile(p)
    assert _load_rc(bbc, p)[0] == bbc.EINVAL
    assert "size" in bbc.load().bbc_last_error().decode()


def test_checksum_of_the_arrays(bbc, tmp_path):
    """A file of the right size whose checksum does not match its arrays is
    refused; the checksum routine itself is pinned to FNV-1a's published
    64-bit test values (the empty input gives the offset basis; one word
    of zeros gives basis * prime mod 2^64)."""
    from helpers import word_fnv64
    assert word_fnv64(b"") == 0xcbf29ce484222325
    assert word_fnv64(b"\0") == (0xcbf29ce484222325 * 0x100000001b3) % (1 << 64)
    assert word_fnv64(b"\x01") == ((0xcbf29ce484222325 ^ 1) * 0x100000001b3) % (1 << 64)
    n, d, nlist, m, bits = 4, 8, 2, 2, 8
    body = 4 * nlist * d + 8 * (nlist + 1) + 8 * n + 4 * m * (1 << bits) * (d // m) + n * m + 4 * n * d
    arrays = np.random.default_rng(0).integers(0, 255, body).astype(np.uint8)
    arrays[4 * nlist * d:4 * nlist * d + 8 * (nlist + 1)] = 0  # list_off all zero: consistent only if checked later
    good = word_fnv64(arrays.tobytes())
    p = tmp_path / "altered.bbc"
    np.concatenate([_header(), arrays, np.array([good ^ 1], "<u8").view(np.uint8)]).tofile(p)
    assert _load_rc(bbc, p)[0] == bbc.EINVAL
    assert "checksum" in bbc.load().bbc_last_error().decode()
