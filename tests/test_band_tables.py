"""The library's host tables of the banded ECS eigen-preconditioner (Sec. III)
against the oracle: the same bands, a complex orthogonal X per band that
reconstructs the oracle's K_l, and the same eigenvalues.  Host-only calls: no
GPU is needed."""
import numpy as np
import pytest

from oracle import banded, contour, tdse

CASES = [(256, 51.2, 18.0, contour.SECS, 0, 0.5), (256, 51.2, 18.0, contour.TFECS, 3, 0.5),
         (96, 19.2, 7.0, contour.SECS, 0, 0.4), (64, 12.8, 4.0, contour.OFF, 2, 0.5)]


@pytest.mark.parametrize("n,L,R0,kind,code,theta", CASES)
def test_library_band_tables_match_the_oracle(n, L, R0, kind, code, theta):
    from paper_1505_06707_amd import sofft
    prob = sofft.problem(n, L, R0=R0, theta=theta, contour=code)
    lam, xr, st, wd = sofft.band_tables(prob, 0)
    ab = banded.AxisBands(tdse.Axis(n, L, kind=kind, R0=R0, theta=theta))
    for b, K in zip(ab.bands, ab.Kl):
        w = len(b)
        assert all(st[i] == b[0] and wd[i] == w for i in b)
        X = xr[b][:, :w]                                       # rows nu, columns local m
        assert np.all(xr[b][:, w:] == 0)
        assert np.max(np.abs(X.T @ X - np.eye(w))) < 1e-10
        scale = max(1.0, np.max(np.abs(K)))
        assert np.max(np.abs(X.T @ np.diag(lam[b]) @ X - K)) < 1e-10 * scale
        key = lambda v: (round(v.real, 6), round(v.imag, 6))
        assert np.allclose(sorted(lam[b], key=key), sorted(ab.lam[b], key=key), rtol=1e-9, atol=1e-9 * scale)


def test_band_tables_reject_a_bad_problem():
    from paper_1505_06707_amd import sofft
    prob = sofft.problem(63, 12.6, R0=4.0)
    with pytest.raises(sofft.SofftError):
        sofft.band_tables(prob, 0)
