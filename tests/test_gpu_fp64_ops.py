"""The library's FP64 division and square root against host IEEE arithmetic (GPU).

The sweeps divide and take square roots of bounded operands (floored
densities and pressures of at least 1e-100, state magnitudes below 1e100)
with their own correctly rounded sequences: the hardware reciprocal
(reciprocal square root) refined by Newton steps on fused multiply-adds and
finished with one exact-remainder correction, without the operand scaling and
special-value handling of a general division.  Every FP64 parity claim rests
on these giving IEEE round-to-nearest results, so they are checked bit for
bit against numpy's IEEE division and square root on about a million seeded
operands over the whole admitted range, its extremes included.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log_uniform(rng, lo, hi, n):
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n) * rng.uniform(1.0, 2.0, n) / 1.5


def _operands():
    rng = np.random.Generator(np.random.PCG64(4141))
    sets = []
    # 1. random magnitudes of both operands over [1e-125, 1e125], random signs
    n = 600_000
    a = _log_uniform(rng, 1e-125, 1e125, n) * rng.choice([-1.0, 1.0], n)
    b = _log_uniform(rng, 1e-125, 1e125, n) * rng.choice([-1.0, 1.0], n)
    sets.append((a, b))
    # 2. the extremes: |a| over [1e-250, 1e250], the quotient kept in range
    n = 300_000
    a = _log_uniform(rng, 1e-250, 1e250, n)
    la = np.log10(a)
    q = 10.0 ** rng.uniform(np.maximum(-250.0, la - 250.0), np.minimum(250.0, la + 250.0))
    sets.append((a, a / q))
    # 3. the floors and the magnitude bound themselves, and their products
    edge = np.array([1e-100, 1e100, 1e-200, 1e200, 1e-250, 1e250, 1e-20, 1e20])
    ea, eb = np.meshgrid(edge, edge)
    ea, eb = ea.ravel(), eb.ravel()
    ok = np.abs(np.log10(ea) - np.log10(eb)) <= 250.0
    sets.append((ea[ok], eb[ok]))
    # 4. structured cases: near 1, all-ones mantissas, exact quotients,
    #    perfect squares, powers of two
    k = np.arange(1, 20_001, dtype=np.float64)
    one_p = 1.0 + k * 2.0 ** -52
    one_m = 1.0 - k * 2.0 ** -53
    sets.append((one_p, one_m))
    sets.append((np.full_like(k, 2.0 - 2.0 ** -52), one_p))
    sets.append((k * 3.0, np.full_like(k, 3.0)))
    sets.append((k * k, k))
    sets.append((2.0 ** rng.integers(-800, 800, 20_000).astype(np.float64),
                 2.0 ** rng.integers(-30, 30, 20_000).astype(np.float64)))
    a = np.concatenate([s[0] for s in sets])
    b = np.concatenate([s[1] for s in sets])
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b)) and np.all(b != 0.0)
    ratio = np.abs(a / b)
    assert ratio.min() >= 1e-251 and ratio.max() <= 1e251
    return a, b


def _ulps(x, y):
    xi = x.view(np.int64)
    yi = y.view(np.int64)
    return np.abs(xi - yi)


def test_division_and_square_root_equal_ieee():
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    a, b = _operands()
    print(f"{a.size} operand pairs", flush=True)
    ta = torch.from_numpy(a).to("cuda")
    tb = torch.from_numpy(b).to("cuda")
    quot = torch.empty_like(ta)
    root = torch.empty_like(ta)
    ppm.ppm_fp64_ops(ta, tb, quot, root)
    torch.cuda.synchronize()
    q = quot.cpu().numpy()
    want_q = a / b
    bad = q != want_q
    assert not bad.any(), (int(bad.sum()), a[bad][:4], b[bad][:4], _ulps(q[bad], want_q[bad])[:4])
    # square root of the positive operands (the sweeps only take roots of
    # positive bounded values)
    ta = torch.from_numpy(np.abs(a)).to("cuda")
    ppm.ppm_fp64_ops(ta, tb, quot, root)
    torch.cuda.synchronize()
    r = root.cpu().numpy()
    want_r = np.sqrt(np.abs(a))
    bad = r != want_r
    assert not bad.any(), (int(bad.sum()), np.abs(a)[bad][:4], _ulps(r[bad], want_r[bad])[:4])


def test_empty_and_invalid_calls():
    import torch
    from paper_1307_2265_amd import ppm
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    ppm.ppm_fp64_ops(z, z, z, z)  # n = 0 launches nothing
    L = ppm.lib()
    assert L.ppm_fp64_ops(None, None, None, None, 5, None) == ppm.PPM_EINVAL
    assert L.ppm_fp64_ops(None, None, None, None, -1, None) == ppm.PPM_EINVAL
