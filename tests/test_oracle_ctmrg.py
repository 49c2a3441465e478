"""Pins of the oracle's CTMRG and readout, independent of the simple update.

* Onsager: the same CTMRG contracting the 2D Ising partition function (one
  tensor per site, bond dimension 2, boundary fixed to + spins) gives the
  exact spontaneous magnetisation (1 - sinh(2 beta)^-4)^(1/8);
* product states: for a random D = 1 state the environment is exact at any
  chi, the readout equals <phi|O|phi>/<phi|phi> and every corner spectrum is
  (1, 0, ...);
* basis independence: rewriting every double-layer leg in the Hermitian
  (real) basis {E_kk, (E_kk'+E_k'k)/sqrt2, i(E_kk'-E_k'k)/sqrt2} and its
  transpose on the opposite end of each bond leaves the corner spectra and the
  readout unchanged, and makes every tensor real (the premise of the device
  path's real arithmetic).
"""
import numpy as np
import pytest

from oracle import ctmrg as ct
from oracle import peps
from oracle.model import Params


def _ising(beta):
    B = np.array([[np.exp(beta), np.exp(-beta)], [np.exp(-beta), np.exp(beta)]])
    lam, U = np.linalg.eigh(B)
    W = (U * np.sqrt(lam)) @ U.T            # symmetric square root
    a = np.einsum("su,sl,sd,sr->uldr", W, W, W, W)
    b = np.einsum("s,su,sl,sd,sr->uldr", np.array([1.0, -1.0]), W, W, W, W)
    return a.astype(complex), b.astype(complex), W


@pytest.mark.parametrize("beta,exact", [(0.5, 0.911319377877), (0.6, 0.973608667440)])
def test_onsager_magnetisation(beta, exact):
    onsager = (1 - np.sinh(2 * beta) ** -4) ** 0.125
    assert abs(onsager - exact) < 1e-11
    a, b, W = _ising(beta)
    lat = {s: a for s in peps.SITES}
    env, it, delta = ct.ctmrg(lat, 32, bvec=W[0].astype(complex), max_iter=200, tol=1e-10)
    assert delta < 1e-10
    for s in peps.SITES:
        E = ct.site_environment(env[s])
        m = (np.sum(E * b) / np.sum(E * a)).real
        assert abs(m - onsager) < 1e-9


def _random_product_state(rng, D, d_A=2):
    p = Params(D=D, chi=max(1, D * D), d_A=d_A)
    st = peps.new_state(p)
    phis = {}
    for s in peps.SITES:
        phi = rng.normal(size=2 * d_A) + 1j * rng.normal(size=2 * d_A)
        g = np.zeros_like(st["gam"][s])
        g[:, 0, 0, 0, 0] = phi
        st["gam"][s] = g
        phis[s] = phi
    return p, st, phis


@pytest.mark.parametrize("D,chi", [(1, 1), (1, 5), (2, 4), (2, 9)])
def test_product_state_exact(D, chi):
    rng = np.random.default_rng(11 + D + chi)
    p, st, phis = _random_product_state(rng, D)
    env, _, _ = ct.ctmrg(ct.double_layers(st), chi, max_iter=3)
    for s in peps.SITES:
        rho = ct.reduced_density_matrix(ct.site_environment(env[s]), ct.absorb_sqrt_lambda(st, s))
        phi = phis[s]
        ref = np.outer(phi, phi.conj()) / np.vdot(phi, phi)
        assert np.max(np.abs(rho - ref)) < 1e-13
    spec = ct.corner_spectra(env, chi)
    assert np.max(np.abs(spec[:, 0] - 1.0)) < 1e-13
    if chi > 1:
        assert np.max(np.abs(spec[:, 1:])) < 1e-13


def hermitian_basis(D):
    """Rows: the D^2 Hermitian matrices H_m flattened over (k, k')."""
    Hs = []
    for k in range(D):
        for kp in range(D):
            H = np.zeros((D, D), dtype=complex)
            if k == kp:
                H[k, k] = 1.0
            elif k < kp:
                H[k, kp] = H[kp, k] = 1 / np.sqrt(2)
            else:
                H[k, kp] = 1j / np.sqrt(2)
                H[kp, k] = -1j / np.sqrt(2)
            Hs.append(H.reshape(-1))
    return np.array(Hs)


def to_real_basis(a, D):
    """up/left legs contract with H_m, down/right legs with H_m^T."""
    U = hermitian_basis(D)
    UT = np.array([u.reshape(D, D).T.reshape(-1) for u in U])
    return np.einsum("wxyz,uw,lx,my,rz->ulmr", a, U, U, UT, UT, optimize=True)


def test_real_basis_invariance():
    rng = np.random.default_rng(3)
    D, chi = 2, 8
    p = Params(D=D, chi=chi)
    st = peps.new_state(p)
    for s in peps.SITES:
        st["gam"][s] = rng.normal(size=st["gam"][s].shape) + 1j * rng.normal(size=st["gam"][s].shape)
    for k in ("lam_h", "lam_v"):
        for s in peps.SITES:
            lam = np.sort(rng.uniform(0.1, 1.0, D))[::-1]
            st[k][s] = lam / np.linalg.norm(lam)
    a = ct.double_layers(st)
    ar = {s: to_real_basis(t, D) for s, t in a.items()}
    for t in ar.values():
        assert np.max(np.abs(t.imag)) < 1e-13 * np.max(np.abs(t))
    env_c, _, _ = ct.ctmrg(a, chi, max_iter=6)
    # the boundary vector vec(I) is the indicator of the diagonal elements in both bases
    bvec = np.array([1.0 if k == kp else 0.0 for k in range(D) for kp in range(D)], dtype=complex)
    env_r, _, _ = ct.ctmrg({s: t.real.astype(complex) for s, t in ar.items()}, chi,
                           bvec=bvec, max_iter=6)
    for s in peps.SITES:
        for k in range(4):
            assert np.max(np.abs(env_r[s]["C"][k].imag)) == 0.0
    sc, sr = ct.corner_spectra(env_c, chi), ct.corner_spectra(env_r, chi)
    # the two runs differ only by rounding: the spread measured here (~1e-10)
    # is the floor any two FP64 implementations of this CTMRG can reach
    assert np.max(np.abs(sc - sr)) < 1e-9


def test_renyi_helper_against_matrix_functions():
    """S_1 = -Tr r log r and S_1/2 = 2 log Tr sqrt(r) through scipy's matrix
    logarithm and square root (a different route than the eigenvalues the
    oracle uses), for random density matrices; pure states give 0, the
    maximally mixed state log d for both orders, and S_1/2 >= S_1."""
    from scipy.linalg import logm, sqrtm

    rng = np.random.default_rng(11)
    for d in (2, 3, 4):
        for _ in range(5):
            X = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
            r = X @ X.conj().T
            r /= np.trace(r).real
            s1, sh = ct.renyi(r)
            assert abs(s1 - float(-np.trace(r @ logm(r)).real)) < 1e-10
            assert abs(sh - float(2 * np.log(np.trace(sqrtm(r)).real))) < 1e-10
            assert sh >= s1 - 1e-12
        v = rng.normal(size=d) + 1j * rng.normal(size=d)
        v /= np.linalg.norm(v)
        assert max(abs(x) for x in ct.renyi(np.outer(v, v.conj()))) < 1e-7
        s1, sh = ct.renyi(np.eye(d) / d)
        assert abs(s1 - np.log(d)) < 1e-12 and abs(sh - np.log(d)) < 1e-12
