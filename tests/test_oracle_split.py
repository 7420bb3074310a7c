"""Error of the split-precision products against FP64, emulated on the CPU.

The split form of the translations stores each FP32 operand x as
hi = bf16(x) and lo = bf16(x - hi) (round to nearest even) and forms a real
product as hi*hi + hi*lo + lo*hi with FP32 accumulation; a single-pass bf16
product uses hi*hi alone.  Both are emulated here with NumPy on the oracle's
own translation matrices D (Sec. 3, Eq. 12) and equivalent sources of a seeded
vector, and compared with the FP64 product: the split form sits near the 2^-16
level of its two-term mantissa (median 5e-6), the single pass near bf16's 2^-9
(median 2.7e-3).  The
GPU parity tests measure the library's split products against the oracle at the
same level (1.6e-7 - 2.6e-6).
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


def cmat(re, im):
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def products(D, S):
    """FP64, bf16x3 and single-pass bf16 forms of D @ S (complex, FP32 inputs)."""
    D32 = D.astype(np.complex64)
    S32 = S.astype(np.complex64)
    exact = D32.astype(np.complex128) @ S32.astype(np.complex128)
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


def test_bf16x3_and_single_pass_errors(ref):
    x = synth.complex_normal(ref.m.n, 40)
    s = ref.upward(x)
    t = ref.t
    errs3, errs1 = [], []
    for l in ref.levels:
        for a in range(0, len(t.boxes[l]), max(1, len(t.boxes[l]) // 8)):
            ka = t.boxes[l][a]
            for b in t.il[l][a][:6]:
                kb = t.boxes[l][b]
                D = ref.D(l, (ka[0] - kb[0], ka[1] - kb[1], ka[2] - kb[2]))
                S = s[l][b].T
                if not np.any(S):
                    continue
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
