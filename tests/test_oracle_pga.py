"""Pins of the oracle's completion by PGA (Alg. 5): the momentum schedule,
degenerate masks, the scalar-tensor case against a textbook FISTA written with
SciPy's DCT, and recovery of a low-L-rank tensor."""
import numpy as np
import pytest
import scipy.fft as sfft

import oracle as o
from paper_2202_02870_amd import workloads as wl


def test_schedule_values():
    betas, mus = o.pga_schedule(5, mu0=2.0, nu=0.5, mu_bar=0.4)
    t = [1.0, 1.0]
    for _ in range(5):
        t.append((1 + np.sqrt(4 * t[-1] ** 2 + 1)) / 2)
    expect = [(t[k - 1] - 1) / t[k] for k in range(1, 6)]
    assert np.allclose(betas, expect, atol=0, rtol=1e-15)
    assert betas[0] == 0.0 and betas[1] == 0.0 and betas[2] > 0
    assert np.allclose(mus, [2.0, 1.0, 0.5, 0.4, 0.4])


def test_all_observed_one_step_is_prox_of_M():
    rng = np.random.default_rng(30)
    M = rng.standard_normal((5, 4, 3))
    mats = o.mats_for(M.shape, ["dct"])
    X, info = o.complete_pga(M, np.ones(M.shape, bool), mats, mu0=0.7, max_iter=1)
    assert np.abs(X - o.svt(M, 0.7, mats)).max() < 1e-14


def test_nothing_observed_stays_zero():
    rng = np.random.default_rng(31)
    M = rng.standard_normal((5, 4, 3))
    mats = o.mats_for(M.shape, ["dct"])
    X, info = o.complete_pga(M, np.zeros(M.shape, bool), mats, mu0=0.7, max_iter=7)
    assert np.abs(X).max() == 0.0
    assert info["crit"] == np.inf


def _fista_l1_dct(m, mask, mu, iters):
    """Textbook FISTA for min mu ||dctn(x)||_1 + 1/2 ||P_Omega(x - m)||^2 (step 1,
    t_0 = t_1 = 1, y = x_k + ((t_{k-1} - 1)/t_k)(x_k - x_{k-1}))."""
    x_prev = np.zeros_like(m)
    x = np.zeros_like(m)
    t_prev, t = 1.0, 1.0
    for _ in range(iters):
        y = x + (t_prev - 1) / t * (x - x_prev)
        g = y - mask * (y - m)
        gh = sfft.dctn(g, type=2, norm="ortho", axes=[2, 3])
        xn = sfft.idctn(np.sign(gh) * np.maximum(np.abs(gh) - mu, 0), type=2, norm="ortho", axes=[2, 3])
        x_prev, x = x, xn
        t_prev, t = t, (1 + np.sqrt(4 * t * t + 1)) / 2
    return x


def test_scalar_tensor_case_is_fista_l1():
    # I1 = I2 = 1: the nuclear norm of a 1x1 slice is |x^_p|, so Alg. 5 is FISTA
    # for an l1-in-DCT-domain completion.
    rng = np.random.default_rng(32)
    m = rng.standard_normal((1, 1, 6, 5))
    mask = rng.random(m.shape) < 0.6
    mats = o.mats_for(m.shape, ["dct", "dct"])
    X, _ = o.complete_pga(m, mask, mats, mu0=0.2, fixed_mu=0.2, max_iter=40)
    assert np.abs(X - _fista_l1_dct(m, mask, 0.2, 40)).max() < 1e-12


def test_fixed_point_residual_decreases():
    p = wl.make_problem((12, 10, 4), 2, 0.6, seed=33, dist="normal", rescale=False)
    mats = o.mats_for(p.shape, ["dct"])
    mu = 0.05
    res = []
    for iters in (20, 200):
        X, _ = o.complete_pga(p.M, p.mask, mats, mu0=mu, fixed_mu=mu, max_iter=iters)
        res.append(o.fro(X - o.svt(np.where(p.mask, p.M, X), mu, mats)))
    assert res[1] < 1e-2 * res[0]


def test_config0_recovery():
    # Low-L-rank recovery (configuration "order-3 32x32x8, rank 3, half observed"):
    # the error is bias-limited at O(tau) and far below the data scale.
    p = wl.config0()
    mats = o.mats_for(p.shape, p.kinds)
    s = p.schedule
    X, info = o.complete_pga(p.M, p.mask, mats, mu0=s["mu0"], fixed_mu=s["fixed_mu"],
                             max_iter=s["max_iter"])
    err = o.rse(X, p.X_true)
    assert err < 0.05
    rho, _ = o.multirank(p.X_true, mats)
    assert np.all(rho == 3)


def test_stopping_rule_gated_until_floor():
    p = wl.make_problem((16, 12, 3, 2), 2, 0.5, seed=34)
    mats = o.mats_for(p.shape, p.kinds)
    sp = wl.pga_schedule_params(p.M, p.mask)
    tr = []
    X, info = o.complete_pga(p.M, p.mask, mats, tol=1e-4, max_iter=150, trace=tr, **sp)
    betas, mus = o.pga_schedule(info["iters"], sp["mu0"], sp["nu"], sp["mu_bar"])
    if info["converged"]:
        assert mus[-1] <= sp["mu_bar"] and tr[-1] <= 1e-4
    assert o.rse(X, p.X_true) < 0.1


def test_metrics():
    a = np.zeros((2, 2, 2))
    b = a.copy()
    b[0, 0, 0] = 0.1
    x = np.ones((2, 2, 2))
    assert abs(o.rse(x + (b - a), x) - 0.1 / np.sqrt(8)) < 1e-15
    assert abs(o.psnr(b, a) - 10 * np.log10(8 / 0.01)) < 1e-12
