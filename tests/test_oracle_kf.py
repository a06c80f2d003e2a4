"""Pins of the oracle's track model and Kalman filter against closed forms,
finite differences, exact recovery, chi^2 statistics and a least-squares fit."""
import math

import numpy as np
import pytest
from scipy.optimize import least_squares

from helix import at_x, hits
from paper_1712_09407_amd import synth

XR = synth.ROW_X.astype(np.float64)


def _cov0():
    return np.diag([0.01, 0.01, 1.0, 1.0, 100.0])


@pytest.mark.parametrize("bz,qpt,sp,tl,dx", [
    (0.5, 1.5, 0.2, 0.3, 1.0253), (0.5, -4.0, -0.4, -0.8, 7.0), (0.5, 0.5, 0.0, 0.0, -3.1),
    (-0.5, 2.0, 0.3, 0.1, 40.0), (0.5, 0.0, 0.25, 0.5, 20.0), (0.0, 3.0, -0.1, 0.2, 11.0),
    (0.5, 9.0, 0.6, 0.0, 1.0253), (0.5, -0.3, -0.7, 0.9, 120.0)])
def test_propagation_matches_closed_form_circle(orc, bz, qpt, sp, tl, dx):
    st = np.array([3.0, -12.0, sp, tl, qpt])
    x1 = 100.0
    ref = at_x(x1, st, x1 + dx, bz)
    res = orc.propagate(x1, st, _cov0(), x1 + dx, bz, max_sinphi=0.999)
    assert res is not None
    assert np.allclose(res[0], ref, rtol=0, atol=1e-12 * max(1.0, abs(dx)))


@pytest.mark.parametrize("bz,qpt,sp,tl,dx", [
    (0.5, 1.5, 0.2, 0.3, 1.0253), (0.5, -4.0, -0.4, -0.8, 7.0), (0.5, 0.7, 0.5, 0.4, -30.0),
    (0.5, 1e-5, 0.1, 0.2, 5.0), (0.5, 8.0, -0.6, 1.1, 2.0)])
def test_jacobian_matches_finite_differences(orc, bz, qpt, sp, tl, dx):
    st = np.array([3.0, -12.0, sp, tl, qpt])
    x1 = 120.0
    _, _, J = orc.propagate(x1, st, _cov0(), x1 + dx, bz, max_sinphi=0.999)
    steps = np.array([1e-4, 1e-4, 1e-6, 1e-6, 1e-5])
    Jn = np.zeros((5, 5))
    for j in range(5):
        e = np.zeros(5)
        e[j] = steps[j]
        fp = orc.propagate(x1, st + e, _cov0(), x1 + dx, bz, 0.999)[0]
        fm = orc.propagate(x1, st - e, _cov0(), x1 + dx, bz, 0.999)[0]
        Jn[:, j] = (fp - fm) / (2 * steps[j])
    scale = np.maximum(np.abs(Jn), 1.0)
    assert np.max(np.abs(J - Jn) / scale) < 1e-6


def test_covariance_is_jcjt(orc):
    st = np.array([1.0, 2.0, 0.3, 0.4, 1.2])
    rng = np.random.default_rng(0)
    A = rng.normal(size=(5, 5))
    cov = A @ A.T + np.eye(5)
    st2, cov2, J = orc.propagate(90.0, st, cov, 95.0, 0.5)
    assert np.allclose(cov2, J @ cov @ J.T, rtol=1e-13, atol=1e-13)


def _true_hits(st0, x, bz):
    y, z = hits(x[0], st0, x, bz)
    return y, z


@pytest.mark.parametrize("bz,st0", [
    (0.5, [2.0, 10.0, 0.15, 0.4, 1.3]), (0.5, [-7.0, -40.0, -0.3, -0.7, -0.6]),
    (0.5, [0.0, 5.0, 0.05, 0.1, 4.5]), (0.5, [1.0, 1.0, 0.2, 0.3, 0.0]),
    (0.0, [4.0, 3.0, 0.1, -0.2, 0.0]), (-0.5, [-3.0, 8.0, -0.05, 0.6, 2.2])])
def test_noiseless_helix_exact_recovery(orc, bz, st0):
    """A track whose hits lie exactly on a helix is recovered to 1e-9."""
    st0 = np.array(st0, np.float64)
    x = XR[10:140]
    y, z = _true_hits(st0, x, bz)
    p = orc.default_params(prior_qpt=100.0)
    st, cov, chi2, ndf = orc.fit_hits(x, y, z, bz, p)
    if bz == 0.0:
        st0 = st0.copy()
        st0[4] = 0.0      # q/pT is not measurable without a field
    assert np.all(np.abs(st - st0) <= 1e-9 * np.maximum(1.0, np.abs(st0)))
    assert chi2 < 1e-12
    assert ndf == 2 * x.shape[0] - 5


def _smeared_fits(orc, n_tracks, sigma, seed, n_hits=159, prm=None):
    rng = np.random.default_rng(seed)
    x = XR[:n_hits]
    p = prm or orc.default_params(sigma_y=sigma, sigma_z=sigma)
    chi2n, pulls = [], []
    for _ in range(n_tracks):
        qpt = rng.choice([-1, 1]) / rng.uniform(1.0, 5.0)   # stays inside |sin phi| < 0.6
        st0 = np.array([rng.uniform(-5, 5), rng.uniform(-50, 50), rng.uniform(-0.3, 0.3),
                        rng.uniform(-0.9, 0.9), qpt])
        y, z = _true_hits(st0, x, 0.5)
        y = y + rng.normal(0, sigma, y.shape)
        z = z + rng.normal(0, sigma, z.shape)
        r = orc.fit_hits(x, y, z, 0.5, p)
        assert r is not None
        st, cov, chi2, ndf = r
        chi2n.append(chi2 / ndf)
        pulls.append((st - st0) / np.sqrt(np.diag(cov)))
    return np.array(chi2n), np.array(pulls)


def test_chi2_per_ndf_is_one_on_smeared_tracks(orc):
    n, ndf = 1500, 2 * 159 - 5
    chi2n, pulls = _smeared_fits(orc, n, 0.1, 1)
    tol = 3.0 * math.sqrt(2.0 / (ndf * n))
    assert abs(chi2n.mean() - 1.0) < tol, (chi2n.mean(), tol)
    # pulls: unbiased, unit width (4 standard errors of the sample mean / width)
    m, s = pulls.mean(axis=0), pulls.std(axis=0)
    assert np.all(np.abs(m) < 4.0 / math.sqrt(n)), m
    assert np.all(np.abs(s - 1.0) < 4.0 / math.sqrt(2 * n)), s


def _kf_vs_lsq_gap(orc, sigma, n_tracks=6, seed=5):
    """Largest |KF - least squares| / sigma_p over a few smeared helices."""
    rng = np.random.default_rng(seed)
    p = orc.default_params(sigma_y=sigma, sigma_z=sigma, prior_sinphi=1e4, prior_tanl=1e4,
                           prior_qpt=1e4)
    x = XR[20:150]
    worst = 0.0
    for _ in range(n_tracks):
        st0 = np.array([rng.uniform(-5, 5), rng.uniform(-50, 50), rng.uniform(-0.2, 0.2),
                        rng.uniform(-0.8, 0.8), rng.choice([-1, 1]) / rng.uniform(0.4, 3.0)])
        y, z = _true_hits(st0, x, 0.5)
        y = y + rng.normal(0, sigma, y.shape)
        z = z + rng.normal(0, sigma, z.shape)
        st, cov, chi2, ndf = orc.fit_hits(x, y, z, 0.5, p)

        def resid(q):
            yy, zz = hits(x[0], q, x, 0.5)
            return np.concatenate([(yy - y) / sigma, (zz - z) / sigma])

        err = np.sqrt(np.diag(cov))
        ls = least_squares(resid, st, x_scale=err, xtol=1e-15, ftol=1e-15, gtol=1e-15,
                           method="lm")
        worst = max(worst, float(np.max(np.abs(st - ls.x) / err)))
    return worst


def test_kalman_tends_to_least_squares_with_diffuse_prior(orc):
    """With a diffuse prior a linear Kalman filter is the weighted least-squares
    fit.  The helix is only mildly non-linear, so the filter must approach an
    independent Gauss-Newton fit of the circle model as the noise shrinks, with
    a gap (linearisation error) that scales like sigma."""
    g2 = _kf_vs_lsq_gap(orc, 1e-2)
    g3 = _kf_vs_lsq_gap(orc, 1e-3)
    assert g3 < 0.02, g3
    assert 5.0 < g2 / g3 < 20.0, (g2, g3)
