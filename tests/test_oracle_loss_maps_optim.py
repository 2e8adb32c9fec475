"""Pins of the oracle's sparse NCC loss, error/age maps and hybrid optimizer
against identities, finite differences, numpy/torch library routines and
closed forms (no GPU)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import loss, maps, optim
from oracle.params import LossParams, OptimParams


# ---------------------------------------------------------------- loss
def test_ncc_of_affine_copy_is_plus_minus_one():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(40, 3))
    lp = LossParams(eps_ncc=0.0)
    assert np.allclose(loss.tile_loss(x, 2.5 * x + 0.1, lp)["ncc"], 1.0)
    assert np.allclose(loss.tile_loss(x, -0.7 * x + 0.9, lp)["ncc"], -1.0)


def test_ncc_gradient_is_n_times_derivative_of_one_minus_ncc():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(25, 3))
    y = rng.uniform(size=(25, 3))
    lp = LossParams()
    tl = loss.tile_loss(x, y, lp)
    h = 1e-7
    for i in (0, 7, 24):
        for ch in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, ch] += h
            xm[i, ch] -= h
            fp = 1 - loss.tile_loss(xp, y, lp)["ncc"][ch]
            fm = 1 - loss.tile_loss(xm, y, lp)["ncc"][ch]
            assert np.isclose(25 * (fp - fm) / (2 * h), tl["gn"][i, ch], rtol=1e-6, atol=1e-8)


def test_ncc_gradient_reduces_to_appendix_formula_without_eps():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(30, 3))
    y = rng.uniform(size=(30, 3))
    tl = loss.tile_loss(x, y, LossParams(eps_ncc=0.0))
    mx, my = x.mean(0), y.mean(0)
    vx, vy = x.var(0), y.var(0)
    appendix = -((y - my) / np.sqrt(vx * vy) - tl["ncc"] * (x - mx) / vx)
    assert np.allclose(tl["gn"], appendix, rtol=1e-10)


def test_charbonnier_gradient_and_lambda_range():
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(16, 3))
    y = rng.uniform(size=(16, 3))
    lp = LossParams(eps_charb=1e-3)
    tl = loss.tile_loss(x, y, lp)
    d = x - y
    assert np.allclose(tl["g1"], d / np.sqrt(d * d + 1e-6))
    assert 0.0 <= tl["lam"] <= 1.0
    assert np.allclose(tl["err"], np.abs(d).sum(1))


def test_full_sparse_loss_gradient_matches_finite_differences():
    """dL/dI of Eq. (full_loss) with the per-tile weights held fixed."""
    rng = np.random.default_rng(4)
    off = np.array([0, 12, 30, 31, 50])               # includes a single-pixel tile
    P = off[-1]
    x = rng.uniform(size=(P, 3))
    y = rng.uniform(size=(P, 3))
    P_step, tiles_step = P + 17, 7                     # other views of the step add to the means
    lp = LossParams()
    out = loss.sparse_loss(x, y, off, P_step, tiles_step, lp)
    f0 = loss.loss_value(x, y, off, P_step, tiles_step, out["lam"], lp)
    assert np.isclose(f0, out["loss_l1"] + out["loss_ncc"], rtol=1e-12)
    h = 1e-7
    for i in (0, 11, 12, 30, 49):
        for ch in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, ch] += h
            xm[i, ch] -= h
            fd = (loss.loss_value(xp, y, off, P_step, tiles_step, out["lam"], lp)
                  - loss.loss_value(xm, y, off, P_step, tiles_step, out["lam"], lp)) / (2 * h)
            assert np.isclose(fd, out["dL"][i, ch], rtol=1e-5, atol=1e-10)


# ---------------------------------------------------------------- maps
def _rne(x: Fraction, mant: int, emin: int) -> Fraction:
    """x rounded to nearest, ties to even, in a binary format with ``mant``
    significand bits and smallest normal exponent ``emin`` (subnormals
    included, no overflow handling), in exact rational arithmetic."""
    if x == 0:
        return Fraction(0)
    sgn = 1 if x > 0 else -1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = Fraction(2) ** (max(e, emin) - (mant - 1))           # spacing at x
    k = a / q
    fl = k.numerator // k.denominator
    rem = k - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sgn * fl * q


def _half_bits(v: Fraction) -> int:
    """Bits of a non-negative value that is exactly a finite half."""
    if v == 0:
        return 0
    e = 30
    while e > 0 and Fraction(2) ** (e - 15) > v:
        e -= 1
    if e <= 0:                                                 # subnormal
        return int(v / Fraction(2) ** -24)
    return (e << 10) | int(v / Fraction(2) ** (e - 15) * 1024 - 1024)


def _half_value(bits: int) -> Fraction:
    e, m = (bits >> 10) & 31, bits & 1023
    return Fraction(m, 1024) * Fraction(2) ** -14 if e == 0 else (1 + Fraction(m, 1024)) * Fraction(2) ** (e - 15)


def _ema_bits(E_bits: int, e: float, beta: float) -> int:
    """Eq. (ema_err) built up from exact rationals: the FP32 constants beta
    and 1 - beta, both products and the sum each rounded to FP32 (24 bits),
    then the result rounded to half (11 bits, subnormals below 2^-14)."""
    b = _rne(Fraction(beta), 24, -126)
    omb = _rne(1 - b, 24, -126)
    t1 = _rne(omb * _half_value(E_bits), 24, -126)
    t2 = _rne(b * Fraction(np.float32(e).item()), 24, -126)
    return _half_bits(_rne(t1 + t2, 11, -14))


def test_ema_rounding_matches_exact_rational_construction():
    """The EMA blend's bits against a construction in exact rationals that
    uses no floating-point conversion: random half maps (subnormals, large
    values) and errors, and crafted ties at beta = 1/2 where E and e are
    neighbouring halves h1 < h2, so the FP32 blend is exactly their midpoint
    and round-to-nearest-even must pick the one with the even significand."""
    rng = np.random.default_rng(11)
    H, W = 6, 40
    E = rng.integers(0, 0x7800, size=(H, W)).astype(np.uint16)           # finite, below 32768
    E[0, :8] = rng.integers(1, 1024, size=8)                              # subnormals
    A = np.zeros((H, W), dtype=np.uint16)
    ys, xs = np.nonzero(np.ones((H, W), bool))
    e = np.abs(rng.normal(0.0, 1.0, size=xs.size)).astype(np.float32)
    e[:10] = rng.uniform(0, 1e-5, size=10).astype(np.float32)
    for beta in (0.4, 0.25):
        En, _ = maps.ema_age_update(E, A, xs, ys, e, beta)
        want = [_ema_bits(int(E[y, x]), float(e[i]), beta) for i, (x, y) in enumerate(zip(xs, ys))]
        assert np.array_equal(En[ys, xs], np.array(want, dtype=np.uint16))
    # ties: E = h1, e = h2 (adjacent halves), beta = 1/2
    h1 = rng.integers(0x0400, 0x7000, size=W).astype(np.uint16)
    E2 = np.tile(h1, (1, 1))
    e2 = (h1 + 1).view(np.float16).astype(np.float32)
    En2, _ = maps.ema_age_update(E2, np.zeros_like(E2), np.arange(W), np.zeros(W, np.int64), e2, 0.5)
    even = np.where(h1 % 2 == 0, h1, h1 + 1)
    assert np.array_equal(En2[0], even)
    assert np.array_equal(En2[0], [_ema_bits(int(h), float(x), 0.5) for h, x in zip(h1, e2)])


def test_ema_and_age_update_closed_form():
    H, W = 8, 12
    rng = np.random.default_rng(5)
    E = rng.uniform(0, 2, size=(H, W)).astype(np.float16)
    A = rng.integers(0, 65536, size=(H, W)).astype(np.uint16)
    A[0, 0] = 65535
    xs = np.array([1, 5, 11])
    ys = np.array([0, 3, 7])
    e = np.array([0.3, 1.7, 0.0], dtype=np.float32)
    En, An = maps.ema_age_update(E.view(np.uint16), A, xs, ys, e, 0.4)
    En = En.view(np.float16)
    expect = [_ema_bits(int(E.view(np.uint16)[y, x]), float(e[i]), 0.4) for i, (x, y) in enumerate(zip(xs, ys))]
    assert np.array_equal(En.view(np.uint16)[ys, xs], np.array(expect, dtype=np.uint16))
    mask = np.ones((H, W), bool)
    mask[ys, xs] = False
    assert np.array_equal(En[mask].view(np.uint16), E[mask].view(np.uint16))
    assert (An[ys, xs] == 0).all()
    assert An[0, 0] == 65535
    assert np.array_equal(An[mask & (A < 65535)], A[mask & (A < 65535)] + 1)


def test_dense_error_init_is_half_of_l1():
    rng = np.random.default_rng(6)
    x = rng.uniform(size=(5, 7, 3)).astype(np.float32)
    y = rng.uniform(size=(3, 5, 7)).astype(np.float32)
    e = maps.dense_error_init(x, y).view(np.float16)
    ref = np.abs(x - np.moveaxis(y, 0, -1)).sum(-1)
    assert np.allclose(e.astype(np.float64), ref, rtol=1e-3)


# ---------------------------------------------------------------- optimizer
def _state(N=64, seed=7):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(59, N))
    g = rng.normal(scale=1e-2, size=(59, N))
    m = rng.normal(scale=1e-2, size=(59, N))
    v = rng.uniform(1e-6, 1e-4, size=(59, N))
    return p, g, m, v


def test_lm_rank_one_matches_sherman_morrison():
    p, g, m, v = _state()
    op = OptimParams(lm_mode=0)
    newp, newm, newv = optim.optimizer_step(p, g, m, v, None, op, step=3)
    lr = op.row_lr()
    for rows in (optim.GEOM_ROWS, optim.APP_ROWS):
        gb = g[rows]
        mb = op.beta1 * m[rows] + (1 - op.beta1) * gb
        vb = op.beta2 * v[rows] + (1 - op.beta2) * gb * gb
        Dinv = 1.0 / (np.sqrt(vb) + op.eps_lm)
        # (D + g g^T)^-1 m = D^-1 m - D^-1 g (g^T D^-1 m) / (1 + g^T D^-1 g)
        a = Dinv * mb
        b = Dinv * gb
        delta = -(a - b * (gb * a).sum(0) / (1 + (gb * b).sum(0)))
        assert np.allclose(newp[rows] - p[rows], lr[rows][:, None] * delta, rtol=1e-9, atol=1e-15)


def test_lm_diag_mode_closed_form():
    p, g, m, v = _state(seed=8)
    op = OptimParams(lm_mode=1)
    newp, newm, newv = optim.optimizer_step(p, g, m, v, None, op, step=2)
    rows = optim.GEOM_ROWS + optim.APP_ROWS
    mb, vb = newm[rows], newv[rows]
    delta = -mb / (g[rows] ** 2 + np.sqrt(vb) + op.eps_lm)
    assert np.allclose(newp[rows] - p[rows], op.row_lr()[rows][:, None] * delta, rtol=1e-12)


def test_adam_rows_match_torch_adam_and_sparse_mask():
    torch = pytest.importorskip("torch")
    p, g, m, v = _state(N=16, seed=9)
    op = OptimParams(lm_mode=2, eps_adam=1e-8)
    touched = np.zeros(16, bool)
    touched[::3] = True
    newp, newm, newv = optim.optimizer_step(p, g, np.zeros_like(m), np.zeros_like(v), touched, op, step=1)
    # torch.optim.Adam, one step from zero moments, per row learning rate
    lr = op.row_lr()
    for row in (0, 4, 7, 10, 12, 20, 58):
        t = torch.tensor(p[row, touched], dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([t], lr=float(lr[row]), betas=(op.beta1, op.beta2), eps=op.eps_adam)
        t.grad = torch.tensor(g[row, touched], dtype=torch.float64)
        opt.step()
        assert np.allclose(newp[row, touched], t.detach().numpy(), rtol=1e-12, atol=1e-15)
    assert np.array_equal(newp[:, ~touched], p[:, ~touched])
    assert (newm[:, ~touched] == 0).all() and (newv[:, ~touched] == 0).all()


# ---------------------------------------------------------------- S-SSIM variant
def _ssim_lp():
    return LossParams(structure="ssim")


def test_ssim_identities_and_closed_forms():
    """Sparse SSIM of one tile: SSIM(x, x) = 1 with zero gradient; symmetric
    in x and y; constant tiles reduce to the luminance term
    (2 a b + C1) / (a^2 + b^2 + C1); y = s x + c (s > 0) makes the
    contrast-structure term (2 s V + C2) / ((1 + s^2) V + C2) with V the
    variance of x; and |SSIM| <= 1."""
    rng = np.random.default_rng(21)
    x = rng.uniform(0.1, 0.9, size=(37, 3))
    s, g = loss.ssim_terms(x, x)
    assert np.allclose(s, 1.0, rtol=0, atol=1e-15) and np.allclose(g, 0.0, atol=1e-13)
    y = rng.uniform(0.0, 1.0, size=(37, 3))
    assert np.allclose(loss.ssim_terms(x, y)[0], loss.ssim_terms(y, x)[0], rtol=1e-14, atol=0)
    a, b = 0.3, 0.7
    s_const = loss.ssim_terms(np.full((20, 3), a), np.full((20, 3), b))[0]
    assert np.allclose(s_const, (2 * a * b + loss.SSIM_C1) / (a * a + b * b + loss.SSIM_C1), rtol=1e-14)
    sc, c = 1.7, -0.2
    y2 = sc * x + c
    mx, my = x.mean(0), y2.mean(0)
    V = x.var(0)
    lum = (2 * mx * my + loss.SSIM_C1) / (mx * mx + my * my + loss.SSIM_C1)
    cs = (2 * sc * V + loss.SSIM_C2) / ((1 + sc * sc) * V + loss.SSIM_C2)
    assert np.allclose(loss.ssim_terms(x, y2)[0], lum * cs, rtol=1e-13)
    for _ in range(20):
        u, v = rng.uniform(-1, 2, size=(2, 15, 3))
        assert (np.abs(loss.ssim_terms(u, v)[0]) <= 1 + 1e-12).all()


def test_ssim_gradient_matches_finite_differences():
    """g_s = n d(1 - SSIM)/dx by central differences, per sample and channel."""
    rng = np.random.default_rng(22)
    x = rng.uniform(0.0, 1.0, size=(23, 3))
    y = rng.uniform(0.0, 1.0, size=(23, 3))
    _, g = loss.ssim_terms(x, y)
    n = x.shape[0]
    h = 1e-6
    for i in range(n):
        for ch in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, ch] += h
            xm[i, ch] -= h
            fd = -(loss.ssim_terms(xp, y)[0][ch] - loss.ssim_terms(xm, y)[0][ch]) / (2 * h)
            assert np.isclose(n * fd, g[i, ch], rtol=1e-6, atol=1e-9)


def test_ssim_sparse_loss_gradient_matches_finite_differences():
    """dL/dI of the S-SSIM loss (lambdas held fixed) by central differences
    of loss_value, and the S-NCC loss differs from it."""
    rng = np.random.default_rng(23)
    tile_off = np.array([0, 9, 9, 30, 41])
    x = rng.uniform(0.0, 1.0, size=(41, 3))
    y = rng.uniform(0.0, 1.0, size=(41, 3))
    lp = _ssim_lp()
    out = loss.sparse_loss(x, y, tile_off, 60, 5, lp)
    assert not np.allclose(out["dL"], loss.sparse_loss(x, y, tile_off, 60, 5)["dL"])
    h = 1e-6
    for i in rng.choice(41, 12, replace=False):
        for ch in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, ch] += h
            xm[i, ch] -= h
            fd = (loss.loss_value(xp, y, tile_off, 60, 5, out["lam"], lp) -
                  loss.loss_value(xm, y, tile_off, 60, 5, out["lam"], lp)) / (2 * h)
            assert np.isclose(fd, out["dL"][i, ch], rtol=1e-5, atol=1e-10)
