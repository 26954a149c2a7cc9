"""Pins of the FP64 oracle's scalar building blocks against things other than
itself: an independent Philox implementation (rocRAND's host engine), 40-digit
quadrature and closed forms (mpmath), exact inversion by bisection, and the
printed quadratic of the paper's Appendix A."""
import os
import shutil
import subprocess
import tempfile

import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 40
HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def rocrand_philox():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rocrand_philox")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "helpers", "rocrand_philox.cpp")],
                   check=True, capture_output=True)

    def run(rows):
        inp = "\n".join(" ".join("%x" % v for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [[int(t, 16) for t in line.split()] for line in out.strip().splitlines()]
    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(ora, rocrand_philox):
    rng = np.random.default_rng(123)
    # rocRAND positions its engine with a 64-bit offset of 4 * (c1:c0) outputs,
    # so c1 stays below 2^30 here; c2, c3 and the key take any value
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF, 0x3FFFFFFF] + [0xFFFFFFFF] * 4, [1, 2, 3, 4, 5, 6]]
    for _ in range(200):
        r = list(map(int, rng.integers(0, 2**32, size=6)))
        r[1] &= 0x3FFFFFFF
        rows.append(r)
    ref = rocrand_philox(rows)
    for r, e in zip(rows, ref):
        assert ora.philox(r[:4], r[4:]) == e


def test_uniform_key_counter_layout(ora, rocrand_philox):
    """u(seed, id, step, purpose, d): counter (id_lo, id_hi, step, purpose<<24 | d/2),
    key (seed_lo, seed_hi); words (r0,r1) for even d, (r2,r3) for odd d; 52 bits."""
    cases = [(0, 0, 0, 1, 0), (7, (1 << 40) + 3, 999, 2, 5), (2**63 + 11, 12345678901, 17, 1, 4),
             (3, (1 << 61) + 5, 2**31 + 9, 2, 33)]
    for seed, pid, step, purpose, d in cases:
        row = [pid & 0xFFFFFFFF, pid >> 32, step, (purpose << 24) | (d >> 1),
               seed & 0xFFFFFFFF, seed >> 32]
        r = rocrand_philox([row])[0]
        a, b = (r[2], r[3]) if d & 1 else (r[0], r[1])
        k = (a << 20) | (b >> 12)
        assert ora.uniform(seed, pid, step, purpose, d) == (k + 0.5) / 2.0**52


def test_uniform_moments(ora):
    u = np.array([ora.uniform(0, i, 3, 2, d) for i in range(4000) for d in range(3)])
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
    assert abs((u ** 2).mean() - 1 / 3) < 4 * np.sqrt(4 / 45 / len(u))
    # no correlation between the two halves of one Philox call
    a = np.array([ora.uniform(5, i, 0, 1, 0) for i in range(4000)])
    b = np.array([ora.uniform(5, i, 0, 1, 1) for i in range(4000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 4 / np.sqrt(4000)


# ---------------------------------------------------------------- Planck
def mp_band(xl, xh):
    f = lambda t: t ** 3 / mp.expm1(t)
    return mp.quad(f, [xl, xh])


def mp_tail(x):
    f = lambda t: t ** 3 / mp.expm1(t)
    return mp.quad(f, [x, x + 10, x + 40, mp.inf])


def test_planck_tail_closed_form_and_quadrature(ora):
    assert ora.planck_tail(0.0) == pytest.approx(float(mp.pi ** 4 / 15), rel=1e-16, abs=0)
    for x in [1e-6, 1e-3, 0.1, 0.5, 1.0, 1.5, 1.999, 2.0, 2.001, 3.0, 7.5, 20.0, 60.0, 300.0]:
        ref = float(mp_tail(x))
        assert ora.planck_tail(x) == pytest.approx(ref, rel=2e-15), x
    assert ora.planck_tail(800.0) == 0.0


def test_planck_head_small_x(ora):
    for x in [1e-8, 1e-4, 0.01, 0.3, 1.0, 1.9999]:
        ref = float(mp.quad(lambda t: t ** 3 / mp.expm1(t), [0, x]))
        assert ora.planck_head(x) == pytest.approx(ref, rel=2e-15), x


@pytest.mark.parametrize("T", [1e-3, 0.05, 0.3, 1.0, 7.0])
def test_phi_group_against_quadrature(ora, T):
    edges = np.geomspace(0.01, 10.0, 11)
    for g in range(10):
        nl, nh = edges[g], edges[g + 1]
        ref = float(T ** 4 * mp_band(mp.mpf(nl) / T, mp.mpf(nh) / T) * 15 / mp.pi ** 4)
        got = ora.phi_group(T, nl, nh, 1.0, 1.0)
        if ref < 1e-300:
            assert got == pytest.approx(ref, abs=1e-300)
        else:
            assert got == pytest.approx(ref, rel=5e-14), (T, g)


def test_phi_sum_is_acT4(ora):
    # the full spectrum carries a c T^4 (Sec. 2.1)
    edges = np.geomspace(1e-7, 2e3, 64)
    for T in [0.5, 1.0, 3.0]:
        tot = sum(ora.phi_group(T, edges[g], edges[g + 1], 0.7, 3.0) for g in range(63))
        assert tot == pytest.approx(0.7 * 3.0 * T ** 4, rel=1e-13)


def test_dphi_matches_finite_difference(ora):
    edges = np.geomspace(0.01, 10.0, 9)
    for T in [0.002, 0.1, 1.0]:
        for g in range(8):
            nl, nh = edges[g], edges[g + 1]
            f = lambda t: float(mp.mpf(t) ** 4 * mp_band(mp.mpf(nl) / t, mp.mpf(nh) / t) * 15 / mp.pi ** 4)
            h = T * 1e-6
            ref = (f(T + h) - f(T - h)) / (2 * h)
            got = ora.dphi_group(T, nl, nh, 1.0, 1.0)
            if abs(ref) < 1e-250:
                continue
            assert got == pytest.approx(ref, rel=1e-8), (T, g)


# ---------------------------------------------------------------- flux coefficients
SVALS = [1e-12, 1e-8, 1e-5, 1e-3, 0.01, 0.3, 0.999, 1.0, 1.001, 1.5, 1.999, 2.0, 2.001, 5.0, 30.0, 1e3, 1e6]


def mp_c4(s):
    s = mp.mpf(s)
    return -mp.expm1(-s) / s


def mp_c2_over_dt(s):
    # Eq. C2Formula with dt = 1 and tau = 1/s:  2 tau^2 (1-e^-s) - tau - tau e^-s
    s = mp.mpf(s)
    tau = 1 / s
    return 2 * tau ** 2 * (-mp.expm1(-s)) - tau - tau * mp.exp(-s)


def test_c4(ora):
    assert ora.coef_c4(0.0) == 1.0
    for s in SVALS:
        assert ora.coef_c4(s) == pytest.approx(float(mp_c4(s)), rel=1e-15), s


def test_w_is_c4_minus_exp(ora):
    assert ora.coef_w(0.0) == 0.0
    for s in SVALS:
        ref = mp_c4(s) - mp.exp(-mp.mpf(s))
        assert ora.coef_w(s) == pytest.approx(float(ref), rel=2e-15), s


def test_c2(ora):
    assert ora.coef_c2_over_dt(0.0) == 0.0
    for s in SVALS:
        assert ora.coef_c2_over_dt(s) == pytest.approx(float(mp_c2_over_dt(s)), rel=4e-15), s
    # limits: thin C2 -> -s dt/6, thick C2 -> -tau (diffusion)
    assert ora.coef_c2_over_dt(1e-9) == pytest.approx(-1e-9 / 6, rel=1e-8)
    assert ora.coef_c2_over_dt(1e8) * 1e8 == pytest.approx(-1.0, rel=1e-7)


# ---------------------------------------------------------------- frequency sampling
def B(nu, T):
    return nu ** 3 / mp.expm1(nu / T)


def test_slope_matches_planck_ratio(ora):
    for (nl, nh, T) in [(1.0, 1.2, 1.0), (0.01, 0.0133, 1.0), (3.0, 4.0, 1.0), (0.5, 0.6, 0.2)]:
        nm = (nl + nh) / 2
        ref = (B(mp.mpf(nh), T) - B(mp.mpf(nl), T)) / B(mp.mpf(nm), T)
        ref = max(-2.0, min(2.0, float(ref)))
        assert ora.freq_slope(nl, nh, T) == pytest.approx(ref, rel=1e-13, abs=1e-15)
    # steep Wien tail (B(mid) underflows): limited, not NaN
    assert ora.freq_slope(5.0, 6.0, 1e-3) == -2.0
    assert ora.freq_slope(0.01, 0.02, 1e-3) == -2.0


def test_sampler_inverts_linear_cdf_by_bisection(ora):
    rng = np.random.default_rng(3)
    for _ in range(300):
        nl = 10 ** rng.uniform(-2, 1)
        nh = nl * rng.uniform(1.01, 3)
        beta = rng.uniform(-2, 2)
        U = rng.uniform(0, 1)
        # exact CDF of the pdf (1 + beta u')/dnu on u' in [-1/2, 1/2]
        G = lambda u: (u + 0.5) + 0.5 * beta * (u * u - 0.25)
        lo, hi = -0.5, 0.5
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if G(mid) < U:
                lo = mid
            else:
                hi = mid
        ref = 0.5 * (nl + nh) + 0.5 * (lo + hi) * (nh - nl)
        assert ora.sample_nu(nl, nh, beta, U) == pytest.approx(ref, abs=1e-14 * nh)


def test_sampler_matches_appendix_A_quadratic(ora):
    """Unclamped case: the root of a nu^2 + b nu + c = 0 with the printed a, b, c."""
    nl, nh, T, eta = mp.mpf("0.35"), mp.mpf("0.5"), mp.mpf("0.3"), mp.mpf("0.37")
    nm = (nl + nh) / 2
    k = (B(nh, T) - B(nl, T)) / (nh - nl)
    Bm = B(nm, T)
    a = k / 2
    b = Bm - k * nm
    c = k * nl * nm - Bm * nl - k / 2 * nl ** 2 - eta * Bm * (nh - nl)
    roots = [(-b + sgn * mp.sqrt(b * b - 4 * a * c)) / (2 * a) for sgn in (1, -1)]
    root = [r for r in roots if nl <= r <= nh]
    assert len(root) == 1
    beta = float(k * (nh - nl) / Bm)
    assert abs(beta) < 2
    got = ora.sample_nu(float(nl), float(nh), beta, float(eta))
    assert got == pytest.approx(float(root[0]), rel=1e-14)


def test_sampler_histogram(ora):
    nl, nh, beta = 1.0, 2.0, -1.3
    rng = np.random.default_rng(11)
    U = rng.uniform(size=200000)
    nu = np.array([ora.sample_nu(nl, nh, beta, u) for u in U])
    assert nu.min() >= nl and nu.max() <= nh
    h, e = np.histogram(nu, bins=20, range=(nl, nh))
    uc = 0.5 * (e[:-1] + e[1:]) - 1.5
    expect = len(U) * (1 + beta * uc) * (e[1] - e[0])
    z = (h - expect) / np.sqrt(expect)
    assert np.max(np.abs(z)) < 5
