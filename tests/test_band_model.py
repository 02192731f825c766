"""The float32 kernel's rounding band (rp_f32_band) against an emulation of
its arithmetic on the CPU, with every rounding taken at its worst:

- u = fl32(U) for the exact scaled difference U = (x - x_p) 2^e (one rounding);
- hi = fp16(u), lo = fp16(u - hi) (round to nearest), FP16 subnormals flushed
  to zero (the matrix unit may flush them);
- the three products hi hi', hi lo', lo hi' of every dimension (exact in FP32)
  summed in FP32 with rounding toward zero, in an adversarial order (the
  largest magnitudes first, so later small terms are truncated away), in
  accumulator chunks of the kernel's length (rp_f32_band reports it), the
  chunk results summed the same way;
- S~ = fl32(fl32(s_i) + fl32(s_j)) - 2 G~ with truncating operations.

On pairs built to stress each term (near-duplicates, cancelling coordinates,
values at the FP16 subnormal edge, wide dynamic ranges, d up to 960) the
emulated error never exceeds c1 s + c2 sqrt(s) + c3 against the canonical FP64
distance (the oracle's).  No GPU is used.
"""
import math

import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(2602)


def _band(d):
    from paper_2602_08097_amd.rp import f32_band

    return f32_band(d)


def _rz32(x):
    """Round float64 values toward zero to float32."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    over = np.abs(f.astype(np.float64)) > np.abs(x)
    f[over] = np.nextafter(f[over], np.float32(0.0))
    return f


def _split(u):
    hi = u.astype(np.float16)
    lo = (u - hi.astype(np.float32)).astype(np.float16)  # u - hi is exact in FP32
    tiny = np.float16(2.0 ** -14)
    hi = np.where(np.abs(hi) < tiny, np.float16(0), hi)
    lo = np.where(np.abs(lo) < tiny, np.float16(0), lo)
    return hi.astype(np.float64), lo.astype(np.float64)


def _emulate(xp, xi, xj, e, chunk):
    """S~(i, j) for a batch of pairs (rows of xi, xj) in the frame of xp."""
    sc = 2.0 ** e
    ui = (xi.astype(np.float64) * sc - xp.astype(np.float64) * sc).astype(np.float32)
    uj = (xj.astype(np.float64) * sc - xp.astype(np.float64) * sc).astype(np.float32)
    hi_i, lo_i = _split(ui)
    hi_j, lo_j = _split(uj)
    d = xi.shape[1]
    total = np.zeros(xi.shape[0], np.float32)
    for c0 in range(0, d, chunk):
        sl = slice(c0, min(d, c0 + chunk))
        terms = np.concatenate([hi_i[:, sl] * hi_j[:, sl], hi_i[:, sl] * lo_j[:, sl],
                                lo_i[:, sl] * hi_j[:, sl]], axis=1)
        order = np.argsort(-np.abs(terms), axis=1, kind="stable")
        terms = np.take_along_axis(terms, order, axis=1)
        acc = np.zeros(xi.shape[0], np.float32)
        for t in range(terms.shape[1]):
            acc = _rz32(acc.astype(np.float64) + terms[:, t])
        total = _rz32(total.astype(np.float64) + acc.astype(np.float64))
    return total


def _check(xp, XI, XJ, label):
    d = XI.shape[1]
    c1, c2, c3, chunk = _band(d)
    worst = 0.0
    for r in range(XI.shape[0]):
        xi, xj = XI[r], XJ[r]
        bound_x = max(np.abs(xi).max(), np.abs(xj).max()) + np.abs(xp).max()
        e = min(100, max(-115, 14 - math.frexp(float(bound_x))[1]))
        si = oracle.sqdist(xp, xi)
        sj = oracle.sqdist(xp, xj)
        if si > sj:
            xi, xj, si, sj = xj, xi, sj, si
        sc2 = 2.0 ** (2 * e)
        G = _emulate(xp, xi[None, :], xj[None, :], e, chunk)[0]
        ssum = _rz32(float(np.float32(si * sc2)) + float(np.float32(sj * sc2)))
        s_t = float(_rz32(float(ssum) - 2.0 * float(G)))
        exact = oracle.sqdist(xi, xj) * sc2
        s = sj * sc2
        E = c1 * s + c2 * math.sqrt(s) + c3
        err = abs(s_t - exact)
        assert err <= E, (label, r, err, E)
        worst = max(worst, err / E)
    return worst


@pytest.mark.parametrize("d", [32, 96, 300, 960])
def test_band_holds_on_random_mixture_pairs(d):
    xp = RNG.standard_normal(d).astype(np.float32)
    XI = (xp + 0.3 * RNG.standard_normal((40, d))).astype(np.float32)
    XJ = (xp + 0.3 * RNG.standard_normal((40, d))).astype(np.float32)
    _check(xp, XI, XJ, "mixture")


@pytest.mark.parametrize("d", [64, 960])
def test_band_holds_on_near_duplicates_and_cancellation(d):
    """S(i, j) much smaller than S(p, j): the relative terms must scale with s,
    not with S(i, j)."""
    xp = RNG.standard_normal(d).astype(np.float32)
    base = (xp + RNG.standard_normal((30, d))).astype(np.float32)
    XI = base
    XJ = (base + 1e-4 * RNG.standard_normal((30, d))).astype(np.float32)
    _check(xp, XI, XJ, "near-duplicate")
    # coordinates of alternating sign and equal magnitude (sums that cancel)
    v = np.where(np.arange(d) % 2 == 0, 1.0, -1.0).astype(np.float32)
    XI = np.stack([xp + v * (1 + 1e-3 * k) for k in range(10)]).astype(np.float32)
    XJ = np.stack([xp - v * (1 - 1e-3 * k) for k in range(10)]).astype(np.float32)
    _check(xp, XI, XJ, "cancelling")


@pytest.mark.parametrize("d", [48, 960])
def test_band_holds_at_the_fp16_subnormal_edge_and_wide_range(d):
    """Scaled differences spanning 2^-30 .. 2^13: many hi / lo parts are FP16
    subnormals (flushed), which the absolute terms c2 sqrt(s) and c3 cover."""
    xp = np.zeros(d, np.float32)
    mags = 2.0 ** RNG.uniform(-30, 13, (40, d))
    XI = (mags * RNG.choice([-1, 1], (40, d))).astype(np.float32)
    XJ = (XI * (1 + 2.0 ** -12 * RNG.standard_normal((40, d)))).astype(np.float32)
    _check(xp, XI, XJ, "wide range")
    XI = (2.0 ** -20 * RNG.standard_normal((20, d))).astype(np.float32)
    XJ = (2.0 ** -20 * RNG.standard_normal((20, d))).astype(np.float32)
    XI[:, 0] = 1.0  # sets the frame so the rest lands near the FP16 subnormal edge
    _check(xp, XI, XJ, "subnormal edge")


def test_band_constants_grow_with_d_and_chunking():
    c_small = _band(96)[:3]
    c_large = _band(960)[:3]
    assert all(a > 0 for a in c_small + c_large)
    assert _band(96)[3] == 96 and _band(960)[3] < 960  # restarted above d = 128
    assert c_large[1] > c_small[1] and c_large[2] > c_small[2]  # sqrt(d) and d terms
