"""Error of the split-precision products against FP64, emulated on the CPU.

The split form of the translations stores each FP32 operand x as
hi = bf16(x) and lo = bf16(x - hi) (round to nearest even) and forms a real
product as hi*hi + hi*lo + lo*hi with FP32 accumulation; a single-pass bf16
product uses hi*hi alone.  Both are emulated here with NumPy on the oracle's
own translation matrices D (Sec. 3, Eq. 12) and equivalent sources of a seeded
vector, and compared with the FP64 product: the split form sits near the 2^-16
level of its two-term mantissa (median 5e-6), the single pass near bf16's 2^-9
(median 2.7e-3).  The fp16 form (11-bit parts, each operand first scaled by a
power of two that puts its largest part below 2^14) sits near 2^-22.  The
GPU parity tests measure the library's split products against the oracle at the
same levels.
"""
import numpy as np
import pytest

import synth
from oracle import nesa


def bf16(a):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def split(a):
    hi = bf16(a)
    lo = bf16(a - hi)
    return hi, lo


def fp16_split(a):
    """hi = fp16(a 2^s), lo = fp16(a 2^s - hi) with one power-of-two scale 2^s
    for the whole array (largest magnitude below 2^14), returned unscaled."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    m = float(np.abs(a).max())
    e = np.frexp(m)[1] if m > 0 else -1000
    s = min(max(14 - e, -120), 120)
    sa = np.ldexp(a, s).astype(np.float32)
    hi = sa.astype(np.float16).astype(np.float32)
    lo = (sa - hi).astype(np.float16).astype(np.float32)
    return np.ldexp(hi.astype(np.float64), -s), np.ldexp(lo.astype(np.float64), -s)


def cmat(re, im):
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def products(D, S, fmt="bf16"):
    """FP64, x3 split and single-pass forms of D @ S (complex, FP32 inputs)."""
    D32 = D.astype(np.complex64)
    S32 = S.astype(np.complex64)
    exact = D32.astype(np.complex128) @ S32.astype(np.complex128)
    if fmt == "fp16":
        # one scale per operand (re and im together), as for a matrix family
        # and a level's sources
        dh, dl = fp16_split(np.concatenate([D32.real, D32.imag]))
        sh, sl = fp16_split(np.concatenate([S32.real, S32.imag]))
        (drh, drl), (dih, dil) = (dh[:len(D32)], dl[:len(D32)]), (dh[len(D32):], dl[len(D32):])
        (srh, srl), (sih, sil) = (sh[:len(S32)], sl[:len(S32)]), (sh[len(S32):], sl[len(S32):])
    else:
        (drh, drl), (dih, dil) = split(D32.real), split(D32.imag)
        (srh, srl), (sih, sil) = split(S32.real), split(S32.imag)
    Dh, Dl = cmat(drh, dih), cmat(drl, dil)
    Sh, Sl = cmat(srh, sih), cmat(srl, sil)
    # real products are exact in FP64 for bf16 operands; the sum is what the
    # FP32 accumulator holds up to its own rounding (far below these errors)
    x3 = Dh @ Sh + Dh @ Sl + Dl @ Sh
    x1 = Dh @ Sh
    return exact, x3, x1


@pytest.fixture(scope="module")
def ref():
    v, t = synth.icosphere(10, 0.5)
    return nesa.NesaOracle(v, t, leaf=0.125, d0=3, tau=1e-8)


def _pairs(ref):
    """(D, S) of a spread of translation pairs over every level."""
    x = synth.complex_normal(ref.m.n, 40)
    s = ref.upward(x)
    t = ref.t
    out = []
    for l in ref.levels:
        for a in range(0, len(t.boxes[l]), max(1, len(t.boxes[l]) // 8)):
            ka = t.boxes[l][a]
            for b in t.il[l][a][:6]:
                kb = t.boxes[l][b]
                D = ref.D(l, (ka[0] - kb[0], ka[1] - kb[1], ka[2] - kb[2]))
                S = s[l][b].T
                if np.any(S):
                    out.append((D, S))
    return out


def test_bf16x3_and_single_pass_errors(ref):
    errs3, errs1 = [], []
    for D, S in _pairs(ref):
        exact, x3, x1 = products(D, S)
        nrm = np.linalg.norm(exact)
        errs3.append(np.linalg.norm(x3 - exact) / nrm)
        errs1.append(np.linalg.norm(x1 - exact) / nrm)
    e3, e1 = max(errs3), max(errs1)
    print("translation products: bf16x3 max rel err %.2e (median %.2e), single-pass bf16 %.2e (median %.2e), "
          "%d products" % (e3, np.median(errs3), e1, np.median(errs1), len(errs3)))
    # each operand keeps about 17 bits (hi + lo), each real product drops only
    # lo * lo (2^-18 relative); sums that cancel raise the relative error of the
    # result: median 5e-6, worst 1.5e-5 here
    assert len(errs3) >= 20
    assert np.median(errs3) < 2 ** -16 and e3 < 4e-5
    assert np.median(errs1) > 100 * np.median(errs3)    # the single pass: about 2^-9
    assert e1 < 2 ** -5


def test_fp16x3_errors(ref):
    """The fp16 split: about 22 bits per operand, the dropped lo*lo term and the
    rounding of lo near 2^-22 relative; sums that cancel raise the relative
    error of a result as for bf16."""
    e16, e3 = [], []
    for D, S in _pairs(ref):
        exact, x16, x16_1 = products(D, S, "fp16")
        _, x3, _ = products(D, S)
        nrm = np.linalg.norm(exact)
        e16.append(np.linalg.norm(x16 - exact) / nrm)
        e3.append(np.linalg.norm(x3 - exact) / nrm)
    print("translation products: fp16x3 max rel err %.2e (median %.2e), bf16x3 median %.2e"
          % (max(e16), np.median(e16), np.median(e3)))
    assert len(e16) >= 20
    # measured: median 8.8e-8, worst 3.7e-7 (bf16x3: median 5.3e-6)
    assert np.median(e16) < 2 ** -22 and max(e16) < 2 ** -20
    assert np.median(e3) > 16 * np.median(e16)      # 3 more bits per part, both parts


def test_fp16_split_scale_and_range():
    """The scale puts the largest part below 2^14 whatever the magnitude, so
    hi, lo and the sum of a real and an imaginary part stay finite fp16
    values, and hi + lo restores each value to about 2^-22 of the largest."""
    for mag in (1e-30, 3e-7, 1.0, 7e4, 1e30):
        a = (synth.complex_normal(257, 3) * mag).astype(np.complex64)
        parts = np.concatenate([a.real, a.imag])
        hi, lo = fp16_split(parts)
        m = np.abs(parts).max()
        assert np.all(np.isfinite(hi)) and np.all(np.isfinite(lo))
        assert np.abs(hi + lo - parts).max() <= 2 ** -22 * m
    z, zl = fp16_split(np.zeros(8, np.float32))
    assert not np.any(z) and not np.any(zl)


def test_bf16_rounding_is_nearest_even():
    a = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5e-3, 3.0e38], dtype=np.float32)
    r = bf16(a)
    assert r[0] == 1.0
    assert r[1] == 1.0                          # tie: rounds to the even mantissa
    assert r[2] == np.float32(1.0 + 4 * 2 ** -8)   # tie: rounds up to even
    assert r[3] == 1.0
    assert abs(r[4] - a[4]) <= 2 ** -9 * abs(a[4])
    assert np.isfinite(r[5])
    hi, lo = split(a[:5])
    assert np.all(np.abs((hi.astype(np.float64) + lo) - a[:5]) <= 2 ** -16 * np.abs(a[:5]))
