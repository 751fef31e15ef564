"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, and rejects bad arguments on the host
before anything is enqueued.  Device pointers here are placeholders that the
library must never dereference on these paths."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", hdr)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(hmm_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def h():
    import paper_2605_29208_amd as h
    return h


def test_exports_every_declared_symbol(h):
    lib = ctypes.CDLL(h.LIB_PATH)
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(h.EXPORTED)


def fake_model(h, n=3, family="gaussian", dim=1, theta=True):
    return h.HmmModelC(n, dim, h.FAMILY[family], 0, 0x1000, 0x2000, 0x3000 if theta else None)


def fake_batch(h, lengths, f64=0):
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)
    b = h.HmmBatchC(len(lengths), 0x4000, offs.ctypes.data_as(ctypes.c_void_p).value, 0x5000, f64, 0)
    return b, offs


def ws_size(h, op, m, b, prec):
    out = ctypes.c_size_t()
    st = h._lib.hmm_workspace_size(h.OP[op], ctypes.byref(m), ctypes.byref(b), h.PREC[prec],
                                   ctypes.byref(out))
    return st, out.value


def test_stats_len(h):
    m = fake_model(h, 3, "gaussian")
    assert h._lib.hmm_stats_len(ctypes.byref(m)) == 1 + 3 + 9 + 3 + 3 * 2
    m = fake_model(h, 8, "gamma")
    assert h._lib.hmm_stats_len(ctypes.byref(m)) == 1 + 8 + 64 + 8 + 8 * 3
    m = fake_model(h, 4, "full", dim=5)
    assert h._lib.hmm_stats_len(ctypes.byref(m)) == 1 + 4 + 16 + 4 + 4 * (5 + 15)
    m = fake_model(h, 0, "gaussian")
    assert h._lib.hmm_stats_len(ctypes.byref(m)) == 0


def test_workspace_size_and_validation(h):
    m = fake_model(h, 8, "gamma")
    b, offs = fake_batch(h, [100, 64, 1])
    st, n = ws_size(h, "estep", m, b, "f32")
    assert st == h.HMM_OK and n > 0
    st, n2 = ws_size(h, "estep", m, b, "plain_f32")
    assert st == h.HMM_OK and n2 > 0
    # zero-length sequence
    b0, _ = fake_batch(h, [5, 0, 3])
    st, _ = ws_size(h, "estep", m, b0, "f32")
    assert st == h.HMM_ERR_ARG and "length" in h.last_error()
    # theta unset
    mu = fake_model(h, 8, "gamma", theta=False)
    st, _ = ws_size(h, "estep", mu, b, "f32")
    assert st == h.HMM_ERR_PARAMS_UNSET
    # bad n_states / family / dim
    for bad in (fake_model(h, 0), fake_model(h, 2000), h.HmmModelC(3, 1, 42, 0, 1, 2, 3),
                fake_model(h, 3, "gaussian", dim=2), fake_model(h, 3, "table", dim=2)):
        st, _ = ws_size(h, "estep", bad, b, "f32")
        assert st == h.HMM_ERR_ARG
    # scaled precisions run the E-step (large-state path) but not Viterbi;
    # state counts above 256 have no batched path
    st, n3 = ws_size(h, "estep", m, b, "bf16_scaled")
    assert st == h.HMM_OK and n3 > 0
    st, _ = ws_size(h, "viterbi", m, b, "f16_scaled")
    assert st == h.HMM_ERR_UNSUPPORTED
    st, _ = ws_size(h, "estep", fake_model(h, 300, "gaussian"), b, "f32")
    assert st == h.HMM_ERR_UNSUPPORTED


def test_chunk_path_workspace_covers_records(h):
    # N <= 8 E-step: one 48-byte transfer-matrix record per lane (8 lanes per
    # chunk of 16 steps, FP32) for every chunk and every superchunk of 16
    # chunks, plus the two boundary vectors per chunk
    m = fake_model(h, 8, "gamma")
    b, offs = fake_batch(h, [4096] * 64)
    st, n = ws_size(h, "estep", m, b, "f32")
    assert st == h.HMM_OK
    C = 64 * (4096 // 16)
    SC = C // 16
    assert n >= (C + SC) * 8 * 48 + 2 * (C + 1) * 8 * 4


def test_calls_reject_small_workspace_on_host(h):
    m = fake_model(h, 3, "gaussian")
    b, offs = fake_batch(h, [10, 20])
    st = h._lib.hmm_estep_stats(ctypes.byref(m), ctypes.byref(b), h.PREC["f32"],
                                ctypes.c_void_p(0x6000), None, None, ctypes.c_void_p(0x7000),
                                16, None)
    assert st == h.HMM_ERR_WORKSPACE
    st = h._lib.hmm_estep_stats(ctypes.byref(m), ctypes.byref(b), h.PREC["f32"], None, None,
                                None, ctypes.c_void_p(0x7000), 1 << 40, None)
    assert st == h.HMM_ERR_ARG   # stats is NULL


def test_default_opts_and_chunk_len(h):
    o = h.HmmMstepOptsC()
    h._lib.hmm_mstep_default_opts(ctypes.byref(o))
    assert o.eps_collapse == 1e-8 and o.ridge == 1e-6 and o.nu_tol == 1e-6 and o.max_iter == 100
    assert h._lib.hmm_set_chunk_len(7) == h.HMM_ERR_ARG
    assert h._lib.hmm_set_chunk_len(16) == h.HMM_OK
    assert h._lib.hmm_set_chunk_len(0) == h.HMM_OK


def test_server_host_validation(h):
    """Serving calls reject bad arguments before touching the device."""
    lib = h._lib
    o = h.hmm_server_default_opts()
    assert o.max_batch >= 1 and 1 <= o.n_streams <= 16 and o.precision == h.PREC["f32"]
    out = ctypes.c_void_p()
    assert lib.hmm_server_create(None, ctypes.byref(out)) == h.HMM_ERR_ARG
    bad = h.hmm_server_default_opts()
    bad.n_streams = 17
    assert lib.hmm_server_create(ctypes.byref(bad), ctypes.byref(out)) == h.HMM_ERR_ARG
    bad = h.hmm_server_default_opts()
    bad.precision = h.PREC["plain_f32"]
    assert lib.hmm_server_create(ctypes.byref(bad), ctypes.byref(out)) == h.HMM_ERR_ARG
    bad = h.hmm_server_default_opts()
    bad.max_batch = 0
    assert lib.hmm_server_create(ctypes.byref(bad), ctypes.byref(out)) == h.HMM_ERR_ARG
    assert lib.hmm_server_destroy(None) == h.HMM_ERR_ARG
    n = ctypes.c_int32()
    assert lib.hmm_server_poll(None, None, 0, 0, ctypes.byref(n)) == h.HMM_ERR_ARG
    rid = ctypes.c_uint64()
    assert lib.hmm_server_submit(None, 0, 0, None, 0, 1, None, ctypes.byref(rid)) == h.HMM_ERR_ARG
    t0 = h.hmm_server_now()
    assert h.hmm_server_now() >= t0


def get_variant(h, m, b, prec):
    v, n = ctypes.c_int32(-9), ctypes.c_int32(-9)
    st = h._lib.hmm_get_variant(ctypes.byref(m), ctypes.byref(b), h.PREC[prec], ctypes.byref(v),
                                ctypes.byref(n))
    assert st == h.HMM_OK, h.last_error()
    return v.value, n.value


def test_variant_counts_and_forcing(h):
    """Each route reports its number of schedule variants; a forced variant is
    clamped to the route's count and -1 returns to the untuned default; the
    workspace size covers every variant of the route."""
    chunk = (fake_model(h, 8, "gamma"), fake_batch(h, [100, 64, 1])[0])
    wave = (fake_model(h, 32, "gaussian"), fake_batch(h, [100, 64, 1])[0])
    block = (fake_model(h, 150, "gaussian"), fake_batch(h, [3000, 64, 1])[0])
    try:
        assert get_variant(h, *chunk, "f32") == (0, 3)
        assert get_variant(h, *chunk, "f64") == (0, 2)
        assert get_variant(h, *wave, "f32") == (0, 4)
        assert get_variant(h, *block, "f64") == (0, 3)
        sizes = []
        for v in (0, 1, 2):
            assert h._lib.hmm_set_variant(v) == h.HMM_OK
            assert get_variant(h, *block, "f32") == (v, 3)
            assert get_variant(h, *chunk, "f64")[0] == min(v, 1)
            assert get_variant(h, *wave, "f32")[0] == v
        assert h._lib.hmm_set_variant(3) == h.HMM_OK
        assert get_variant(h, *wave, "f32") == (3, 4)
        assert get_variant(h, *block, "f32") == (2, 3)
        assert h._lib.hmm_set_variant(-1) == h.HMM_OK
        assert get_variant(h, *block, "f32") == (0, 3)
        assert h._lib.hmm_set_variant(-2) == h.HMM_ERR_ARG
        st, full = ws_size(h, "estep", *block, "f32")
        assert st == h.HMM_OK
        for v in (0, 1, 2):
            h._lib.hmm_set_variant(v)
            # the size does not depend on the forced variant: it covers them all
            assert ws_size(h, "estep", *block, "f32") == (h.HMM_OK, full)
            sizes.append(full)
    finally:
        h._lib.hmm_set_variant(-1)
