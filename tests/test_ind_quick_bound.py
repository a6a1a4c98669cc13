"""CPU check of the quick Ind test's reasoning (the GPU's first test of a depth-order pair).

The identity bound of d_i - d_j with D = uw_i - uw_j and the depth row of A in
mid-radius form (Zm, Zr; lower coefficients Zm - Zr, upper Zm + Zr, not necessarily
ordered) has lower end (m_P - r_P) - sum_k |m_k - r_k| and upper end (m_P + r_P) +
sum_k |m_k + r_k|, m = D Zm, r = |D| Zr.  The quick test compares q = D Zm[:, P] with
sum_l |D_l| Zq_l, Zq_l = R_l + 2^-45 (|Zm[l, P]| + R_l), R_l = |Zr[l, P]| +
sum_k (|Zm[l, k]| + |Zr[l, k]|).  Wherever it decides, the identity bound must decide the
same way (evaluated here in FP64 in the GPU's order), on random forms of realistic and
adversarial magnitudes, with negative "radii" included; and summing the radii with their
signs instead must be able to disagree (the mistake a first version made).
"""
import numpy as np

P = 6


def _identity(D, Zm, Zr):
    mid = np.zeros(P + 1)
    rad = np.zeros(P + 1)
    for l in range(3):
        mid = D[l] * Zm[l] + mid
        rad = abs(D[l]) * Zr[l] + rad
    lo = (mid[P] - rad[P]) - np.abs(mid[:P] - rad[:P]).sum()
    hi = (mid[P] + rad[P]) + np.abs(mid[:P] + rad[:P]).sum()
    return 1 if lo > 0 else (0 if hi <= 0 else 2)


def _quick(D, Zm, Zr, signed=False):
    if signed:
        R = Zr[:, P] + (np.abs(Zm[:, :P]) + Zr[:, :P]).sum(1)
    else:
        R = np.abs(Zr[:, P]) + (np.abs(Zm[:, :P]) + np.abs(Zr[:, :P])).sum(1)
    Zq = R + 2.0 ** -45 * (np.abs(Zm[:, P]) + R)
    qc = 0.0
    qr = 0.0
    for l in range(3):
        qc = D[l] * Zm[l, P] + qc
        qr = abs(D[l]) * Zq[l] + qr
    if qc - qr > 0:
        return 1
    if qc + qr < 0:
        return 0
    return None


def _forms(rng, scale_coef, scale_rad):
    Zm = np.concatenate([rng.normal(size=(3, P)) * scale_coef, rng.normal(size=(3, 1))], 1)
    Zr = rng.normal(size=(3, P + 1)) * scale_rad
    return Zm, Zr


def test_quick_decisions_are_the_identity_bounds():
    rng = np.random.default_rng(0)
    fired = 0
    for it in range(300):
        Zm, Zr = _forms(rng, rng.choice([1e-3, 1e-2, 1e-1]), rng.choice([1e-4, 1e-3, 1e-2]))
        for _ in range(200):
            D = rng.normal(size=3) * rng.choice([1e-6, 1e-3, 1e-1, 1.0, 30.0])
            q = _quick(D, Zm, Zr)
            if q is not None:
                fired += 1
                assert q == _identity(D, Zm, Zr)
    assert fired > 20000          # the test decides most pairs of such forms


def test_near_ties_and_large_means():
    """Pairs whose identity bound sits within rounding of zero: the quick test leaves them."""
    rng = np.random.default_rng(1)
    for _ in range(2000):
        Zm, Zr = _forms(rng, 1e-2, 1e-3)
        base = rng.normal(size=3) * 100.0
        # D nearly orthogonal to the nominal depth row: q close to 0
        m = Zm[:, P]
        d = rng.normal(size=3)
        d -= (d @ m) / (m @ m) * m
        D = (base + d * 1e-9) - base
        q = _quick(D, Zm, Zr)
        if q is not None:
            assert q == _identity(D, Zm, Zr)


def test_signed_radii_would_be_wrong():
    rng = np.random.default_rng(2)
    wrong = 0
    for _ in range(200):
        Zm, Zr = _forms(rng, 1e-2, 3e-3)
        for _ in range(100):
            D = rng.normal(size=3) * rng.choice([1e-3, 1e-1, 1.0])
            q = _quick(D, Zm, Zr, signed=True)
            wrong += q is not None and q != _identity(D, Zm, Zr)
    assert wrong > 0
