"""Arithmetic facts the kernels rely on, checked on the CPU.

The FP64 refinement of extreme GGN weights splits a pixel index into row and column and reduces
twiddle indices modulo a probe side n <= 256 without an integer division: every operand v it
divides is a pixel index or a product of two indices below 256, so 0 <= v < 65536, and it takes
the truncated float product fl(fl(v) * fl(1 / n)), then corrects the remainder by one step.
That is exact only if the float quotient is never more than one away from the true one; this
checks it for every operand and every side."""
import numpy as np


def test_float_reciprocal_quotient_is_within_one():
    v = np.arange(0, 256 * 256, dtype=np.int64)
    vf = v.astype(np.float32)
    for n in range(1, 257):
        inv = np.float32(1.0) / np.float32(n)
        q = np.trunc(vf * inv).astype(np.int64)
        exact = v // n
        assert np.all(np.abs(q - exact) <= 1), n
        # the kernel's one-step corrections give the exact quotient and remainder
        r = v - q * n
        qc = np.where(r < 0, q - 1, np.where(r >= n, q + 1, q))
        rc = np.where(r < 0, r + n, np.where(r >= n, r - n, r))
        assert np.array_equal(qc, exact) and np.array_equal(rc, v - exact * n), n
