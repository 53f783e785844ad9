"""sgm_block_orth_noalloc (the block orthogonalisation whose scratch is the
library's static device array, for callers that cannot allocate) against
sgm_block_orth (the same kernels on a caller workspace): two calls in a
row on one GPU, the second with a smaller block, in float64 and float32.
The accepted size must be equal and Q_k, R(1:i, k), R(k, k) equal to
rounding (both run the same kernels; with the same row-chunk counts the
sums are the same, so they are expected bitwise equal here)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(n, i, s, seed, dtype):
    rng = np.random.default_rng(seed)
    Qi, _ = np.linalg.qr(rng.standard_normal((n, i)))
    V = Qi @ rng.standard_normal((i, s)) + rng.standard_normal((n, s))
    ld = ((n + 63) // 64) * 64
    buf = np.zeros((i + s, ld), dtype=dtype)
    buf[:, :n] = np.concatenate([Qi, V], 1).T
    return buf, ld


def _both(lib, torch, n, i, s, seed, precision):
    dtype = np.float32 if precision == "fp32_ir" else np.float64
    buf, ld = _case(n, i, s, seed, dtype)
    q1 = torch.tensor(buf.ravel(), device="cuda")
    q2 = q1.clone()
    ref = lib.block_orth(q1, n, ld, i, s, precision=precision)
    got = lib.block_orth_noalloc(q2, n, ld, i, s, precision=precision)
    return ref, got, q1.cpu().numpy(), q2.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_noalloc_block_orth_matches_workspace_variant(lib, precision):
    import torch
    tol = 1e-12 if precision == "fp64" else 1e-5
    # the second call is smaller than the first: the static scratch keeps
    # the first call's contents, which must not leak into the second
    for (n, i, s, seed) in ((9001, 97, 32, 1), (3001, 17, 8, 2),
                            (5000, 1, 1, 3)):
        ref, got, qa, qb = _both(lib, torch, n, i, s, seed, precision)
        p = ref[0]
        assert got[0] == p == s
        assert np.abs(qb - qa).max() <= tol
        for a, b in zip(ref[1:], got[1:]):
            assert np.abs(b[:, :p] - a[:, :p]).max() <= tol * max(
                1.0, np.abs(a).max())
        print(f"{precision} n={n} i={i} s={s}: bitwise equal "
              f"{np.array_equal(qa, qb) and np.array_equal(ref[1], got[1])}")


def test_noalloc_rejects_blocks_beyond_its_scratch(lib):
    import torch
    q = torch.zeros(64 * 300, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SgmError, match="s <= 64"):
        lib.block_orth_noalloc(q, 64, 64, 8, 65)
    with pytest.raises(lib.SgmError, match="i \\+ s <= 256"):
        lib.block_orth_noalloc(q, 64, 64, 200, 60)
