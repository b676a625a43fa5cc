"""Double-precision division and square root on the GPU round exactly like
the host's (IEEE 754, round to nearest even).

The set-defining predicates of the doublet and link steps use + - * / and
sqrt in double on both the oracle and the GPU; + - * are single correctly
rounded instructions on gfx950, while / and sqrt are instruction sequences
chosen by the compiler.  A test kernel built with the library's flags
(tests/native/fp64_ops.hip) computes a / b and sqrt(a) for 1.0e8 seeded
inputs; every result must equal numpy's bit for bit.
"""
import ctypes as ct
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CHUNK = 1 << 24
N_CHUNKS = 6          # 1.007e8 inputs


def _lib():
    path = os.path.join(os.path.dirname(__file__), "native", "libfp64ops.so")
    if not os.path.exists(path):
        pytest.fail("tests/native/libfp64ops.so is not built (run __graft_entry__.build())")
    L = ct.CDLL(path)
    L.fp64_div_sqrt.restype = ct.c_int
    L.fp64_div_sqrt.argtypes = [ct.c_void_p] * 4 + [ct.c_int64, ct.c_void_p]
    return L


def _doubles(rng, n, exp_lo, exp_hi):
    """Finite doubles with random sign and mantissa and a biased exponent
    uniform in [exp_lo, exp_hi] (0 = subnormal)."""
    mant = rng.integers(0, 1 << 52, size=n, dtype=np.uint64)
    exp = rng.integers(exp_lo, exp_hi + 1, size=n, dtype=np.uint64)
    sign = rng.integers(0, 2, size=n, dtype=np.uint64)
    bits = (sign << np.uint64(63)) | (exp << np.uint64(52)) | mant
    v = bits.view(np.float64)
    v[v == 0] = 1.0
    return v


def _inputs(c, rng):
    if c < 2:       # the whole normal range: quotients over- and underflow
        return _doubles(rng, CHUNK, 1, 2046), _doubles(rng, CHUNK, 1, 2046)
    if c < 4:       # the magnitudes of hit coordinates and their products
        a = np.exp(rng.uniform(np.log(1e-6), np.log(1e6), CHUNK)) * rng.choice([-1.0, 1.0], CHUNK)
        b = np.exp(rng.uniform(np.log(1e-6), np.log(1e6), CHUNK)) * rng.choice([-1.0, 1.0], CHUNK)
        return a, b
    if c == 4:      # subnormal and tiny operands
        return _doubles(rng, CHUNK, 0, 60), _doubles(rng, CHUNK, 0, 1100)
    # exact quotients and roots (integers, squares), and neighbours of them
    k = rng.integers(1, 1 << 26, CHUNK).astype(np.float64)
    m = rng.integers(1, 1 << 26, CHUNK).astype(np.float64)
    a = k * m
    a = np.where(rng.uniform(size=CHUNK) < 0.5, a, np.nextafter(a, np.inf))
    return a, m


def test_fp64_division_and_sqrt_round_like_the_host():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = _lib()
    rng = np.random.Generator(np.random.PCG64(64))
    stream = torch.cuda.current_stream().cuda_stream
    bad_q = bad_r = total = 0
    for c in range(N_CHUNKS):
        a, b = _inputs(c, rng)
        da = torch.from_numpy(a).cuda()
        db = torch.from_numpy(b).cuda()
        q = torch.empty_like(da)
        r = torch.empty_like(da)
        absa = torch.from_numpy(np.abs(a)).cuda()
        assert L.fp64_div_sqrt(da.data_ptr(), db.data_ptr(), q.data_ptr(), r.data_ptr(), CHUNK, stream) == 0
        q_host = q.cpu().numpy()
        assert L.fp64_div_sqrt(absa.data_ptr(), db.data_ptr(), q.data_ptr(), r.data_ptr(), CHUNK, stream) == 0
        r_host = r.cpu().numpy()
        with np.errstate(over="ignore", under="ignore"):
            want_q = a / b
        want_r = np.sqrt(np.abs(a))
        bad_q += int(np.sum(q_host.view(np.int64) != want_q.view(np.int64)))
        bad_r += int(np.sum(r_host.view(np.int64) != want_r.view(np.int64)))
        total += CHUNK
    assert total >= 100_000_000
    assert bad_q == 0 and bad_r == 0, (bad_q, bad_r)
