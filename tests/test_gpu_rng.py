"""Pin of the oracle's Philox4x32-10 against an independent implementation:
rocRAND's PHILOX4_32_10 generator (run as a library on the GPU).  With
seed s its output stream is, word by word, Philox4x32-10 with key
(s_lo, s_hi) applied to the 128-bit counters 0, 1, 2, ... (Salmon et al.,
SC'11, the same construction the oracle follows)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROCRAND_PHILOX = 404


def test_oracle_philox_matches_rocrand(oracle_lib):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    try:
        rr = ctypes.CDLL("/opt/rocm/lib/librocrand.so")
    except OSError:
        pytest.skip("rocRAND not installed")
    n = 4 * 4096
    for seed in (0x0123456789ABCDEF, 1, 0xDEADBEEF):
        gen = ctypes.c_void_p()
        assert rr.rocrand_create_generator(ctypes.byref(gen), ROCRAND_PHILOX) == 0
        assert rr.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        out = torch.zeros(n, dtype=torch.int32, device="cuda")
        assert rr.rocrand_generate(gen, ctypes.c_void_p(out.data_ptr()), ctypes.c_size_t(n)) == 0
        torch.cuda.synchronize()
        rr.rocrand_destroy_generator(gen)
        got = out.cpu().numpy().view(np.uint32).reshape(-1, 4)
        key = (seed & 0xFFFFFFFF, seed >> 32)
        for i in list(range(64)) + list(range(4096 - 64, 4096)):
            ref = oracle_lib.philox((i, 0, 0, 0), key)
            assert (ref == got[i]).all(), (hex(seed), i, [hex(x) for x in ref], [hex(x) for x in got[i]])


def test_oracle_philox_stream_matches_rocrand_on_1e8_counters(oracle_lib):
    """The whole stream, word by word, over 1e8 consecutive counters (ten
    chunks of 1e7; rocRAND continues its stream from call to call)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    try:
        rr = ctypes.CDLL("/opt/rocm/lib/librocrand.so")
    except OSError:
        pytest.skip("rocRAND not installed")
    seed = 0x9E3779B97F4A7C15
    key = (seed & 0xFFFFFFFF, seed >> 32)
    chunk, nchunks = 10_000_000, 10
    gen = ctypes.c_void_p()
    assert rr.rocrand_create_generator(ctypes.byref(gen), ROCRAND_PHILOX) == 0
    try:
        assert rr.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        out = torch.empty(4 * chunk, dtype=torch.int32, device="cuda")
        for c in range(nchunks):
            assert rr.rocrand_generate(gen, ctypes.c_void_p(out.data_ptr()), ctypes.c_size_t(4 * chunk)) == 0
            torch.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint32).reshape(-1, 4)
            ref = oracle_lib.philox_stream(key, c * chunk, chunk)
            bad = np.flatnonzero((got != ref).any(axis=1))
            assert bad.size == 0, (c, int(bad[0]) if bad.size else None)
            print(f"[gpu-test] philox chunk {c}: {chunk} counters equal", flush=True)
    finally:
        rr.rocrand_destroy_generator(gen)
