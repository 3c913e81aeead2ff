"""Pins of the stored oracle references under tests/golden (each written from
the oracle alone by the script beside it): the dense FP64 PMCHWT solution of
the 15,360-unknown sphere scatters like the Mie series of the same sphere
within the discretisation error of an s = 4 icosphere, and its cuts meet where
they must (theta = 0 and 180 deg lie on both planes); the coated-sphere sweep
against the coated series and its symmetry; the ellipsoid's cuts against the
body's mirror symmetry."""

import os

import numpy as np

from oracle import mie

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sphere15360_rcs.txt")


def _db(s, ref):
    floor = 1e-3 * ref.max()
    d = np.abs(10 * np.log10((s + floor) / (ref + floor)))
    return float(np.sqrt(np.mean(d ** 2))), float(d.max())


def test_stored_oracle_rcs_against_mie():
    d = np.loadtxt(GOLDEN)
    assert d.shape == (181, 3)
    th = np.deg2rad(d[:, 0])
    mE, mH = mie.sphere_rcs(2.0, 2.56, th)
    rE, xE = _db(d[:, 1], mE)
    rH, xH = _db(d[:, 2], mH)
    # s = 4: 0.3 / 1.2 dB RMS (s = 5 on the GPU gives 0.12 / 0.43, converging)
    assert rE < 0.5 and rH < 1.5
    assert xE < 2.0 and xH < 4.0
    # forward (theta = 180 deg for incidence along -z) and backward directions
    # are on both cuts: the two polarised cuts agree there
    for i in (0, 180):
        assert abs(10 * np.log10(d[i, 1] / d[i, 2])) < 0.05
    # the forward lobe dominates
    assert np.argmax(d[:, 1]) == 180 and np.argmax(d[:, 2]) == 180


def test_stored_coated_sphere_sweep_against_mie_and_symmetry():
    # tests/golden/coated19200_rcs.txt: the oracle's dense LU solutions of the
    # coarse coated sphere (core s = 3, shell s = 4) for 64 incidences.  The
    # facets are coarse (core edge ~ interior wavelength / 1.8), so the check
    # against the Aden-Kerker series is loose; the sweep must be consistent:
    # incidence from theta_i on a sphere scatters the cut of incidence 0
    # rotated by theta_i (up to facetting), and every cut is positive.
    path = os.path.join(os.path.dirname(__file__), "golden", "coated19200_rcs.txt")
    d = np.loadtxt(path)
    assert d.shape == (181, 65) and np.all(d[:, 1:] > 0)
    th = np.deg2rad(d[:, 0])
    mE, _ = mie.coated_sphere_rcs(1.5, 6 - 0.5j, 2.5, 2.56, th)
    rms, mx = _db(d[:, 1], mE)
    assert rms < 0.25 and mx < 0.6
    # backscatter (theta = theta_i) is the same for every incidence on a sphere
    back = np.array([d[int(round(180.0 * i / 63)), 1 + i] for i in range(64)])
    assert np.std(10 * np.log10(back)) < 0.15


def test_stored_ellipsoid_rcs_symmetry_and_forward_lobe():
    # tests/golden/ellipsoid20_rcs.txt (dense-LU JMCFIE solutions of ellipsoid
    # 20 of the batch, written by tests/golden/make_ellipsoid_rcs.py from the
    # oracle alone).  The ellipsoid is symmetric under z -> -z, so the cut of
    # the incidence from theta equals, mirrored in theta, the cut of the
    # incidence from 180 deg - theta; and for incidence along -z the
    # forward direction (theta = 180 deg) carries the largest lobe
    d = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "ellipsoid20_rcs.txt"))
    assert d.shape == (181, 9)
    assert np.allclose(d[:, 0], np.arange(181.0))
    cuts = d[:, 1:]
    assert np.all(np.isfinite(cuts)) and np.all(cuts > 0)
    for i in range(4):
        assert np.allclose(cuts[:, i], cuts[::-1, 7 - i], rtol=1e-8, atol=0)
    assert np.argmax(cuts[:, 0]) == 180 and np.argmax(cuts[:, 7]) == 0
    # incidences at different angles scatter differently (no repeated column)
    assert np.min([np.abs(cuts[:, i] - cuts[:, i + 1]).max() / cuts[:, i].max() for i in range(7)]) > 1e-2
