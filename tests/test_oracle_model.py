"""Pins of the oracle's local space, bond Hamiltonian and gates.

* gates: unitary, G(tau) G(-tau) = 1, equal to the exponential built from an
  eigen-decomposition (a different method from the oracle's expm);
* Hamiltonian matrix elements enumerated by brute force from Eq. (Hori) and
  Eq. (Hanc) with S = sigma/2;
* dilation identity (the readout equation of "Set up for iPEPS"): exact
  diagonalisation of the dilated cluster (physical + auxiliary spins, fields
  split 1/4 per bond) from Néel ⊗ |+> gives the same occupations as the
  explicit average over all 2^N binary field configurations of the
  spin-1/2 XXZ cluster, on 2x2 and 4x2 tori.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import model


@pytest.mark.parametrize("d_A", [2, 3])
def test_gate_unitary_and_inverse(d_A):
    p = model.Params(D=2, chi=4, J=1.0, V=0.7, W=3.0, d_A=d_A)
    for layer in range(4):
        G = p.layer_gate(layer, 0.05)
        I = np.eye(G.shape[0])
        assert np.max(np.abs(G.conj().T @ G - I)) < 1e-14
        assert np.max(np.abs(p.layer_gate(layer, 0.05) @ p.layer_gate(layer, -0.05) - I)) < 1e-14


def test_gate_matches_eigendecomposition():
    h = model.bond_hamiltonian(1.3, -0.4, 2.5, 0.25, 2)
    lam, U = np.linalg.eigh(h)
    for tau in (0.01, 0.05, 0.5):
        ref = (U * np.exp(-1j * tau * lam)) @ U.conj().T
        assert np.max(np.abs(model.gate(h, tau) - ref)) < 1e-14


@pytest.mark.parametrize("d_A", [2, 3, 5])
def test_bond_hamiltonian_elements(d_A):
    J, V, W, w = 0.9, 1.7, 4.0, 0.25
    h = model.bond_hamiltonian(J, V, W, w, d_A)
    d = 2 * d_A
    z = [1 - 2 * a / (d_A - 1) for a in range(d_A)]
    sz = [0.5, -0.5]
    for si, sj, ti, tj in itertools.product(range(d), repeat=4):
        pi, ai = divmod(si, d_A)
        pj, aj = divmod(sj, d_A)
        qi, bi = divmod(ti, d_A)
        qj, bj = divmod(tj, d_A)
        val = 0.0
        if (ai, aj) == (bi, bj):
            if (pi, pj) == (qi, qj):
                val = V * sz[pi] * sz[pj] + w * W * (sz[pi] * z[ai] + sz[pj] * z[aj])
            elif (pi, pj) == (qj, qi) and pi != pj:
                val = J / 2.0
        assert abs(h[si * d + sj, ti * d + tj] - val) < 1e-15


# ------------------------------------------------------------------ dilation identity
def _torus_bonds(Lx, Ly):
    """Each site's right and down bond (with multiplicity on thin tori)."""
    idx = lambda x, y: (y % Ly) * Lx + (x % Lx)
    bonds = []
    for y in range(Ly):
        for x in range(Lx):
            bonds.append((idx(x, y), idx(x + 1, y)))
            bonds.append((idx(x, y), idx(x, y + 1)))
    return bonds, idx


def _embed_two(op2, i, j, N, dloc):
    """Sparse operator acting with a two-site matrix on sites i < or > j."""
    # build via permutation of a dense-on-two-sites kron
    if i > j:
        perm = np.arange(dloc * dloc).reshape(dloc, dloc).T.reshape(-1)
        op2 = op2[np.ix_(perm, perm)]
        i, j = j, i
    left = sp.identity(dloc ** i, format="csr")
    mid = sp.identity(dloc ** (j - i - 1), format="csr")
    right = sp.identity(dloc ** (N - j - 1), format="csr")
    # op2 acts on (i, j) with identity in between: write as sum of products
    op4 = op2.reshape(dloc, dloc, dloc, dloc)
    out = None
    for a, b, c, e in itertools.product(range(dloc), repeat=4):
        v = op4[a, b, c, e]
        if v == 0:
            continue
        ei = sp.csr_matrix(([1.0], ([a], [c])), shape=(dloc, dloc))
        ej = sp.csr_matrix(([1.0], ([b], [e])), shape=(dloc, dloc))
        term = v * sp.kron(sp.kron(sp.kron(sp.kron(left, ei), mid), ej), right)
        out = term if out is None else out + term
    return out.tocsr()


def _embed_one(op1, i, N, dloc):
    return sp.kron(sp.kron(sp.identity(dloc ** i), sp.csr_matrix(op1)),
                   sp.identity(dloc ** (N - i - 1))).tocsr()


def _evolve(H, psi0, times):
    out = []
    for t in times:
        if H.shape[0] <= 512:
            out.append(scipy.linalg.expm(-1j * t * H.toarray()) @ psi0)
        else:
            out.append(spla.expm_multiply(-1j * t * H, psi0))
    return out


@pytest.mark.parametrize("Lx,Ly,d_A", [(2, 2, 2), (4, 2, 2), (2, 2, 3)])
def test_dilation_identity(Lx, Ly, d_A):
    """Dilated dynamics = average over all d_A^N explicit field
    configurations (fields W z, z on d_A equally spaced levels in [-1, 1])."""
    J, V, W = 1.0, 1.0, 2.0
    times = [0.3, 1.1]
    bonds, idx = _torus_bonds(Lx, Ly)
    N = Lx * Ly
    neel = [0 if (x + y) % 2 == 0 else 1 for y in range(Ly) for x in range(Lx)]
    # --- dilated system through the oracle's bond Hamiltonian
    d = 2 * d_A
    hb = model.bond_hamiltonian(J, V, W, 0.25, d_A)
    H = None
    for (i, j) in bonds:
        t = _embed_two(hb, i, j, N, d)
        H = t if H is None else H + t
    plus = np.ones(d_A) / np.sqrt(d_A)
    psi0 = np.array([1.0])
    for s in range(N):
        loc = np.zeros(d)
        loc[neel[s] * d_A:(neel[s] + 1) * d_A] = plus
        psi0 = np.kron(psi0, loc)
    n_op = model.local_operators(d_A)["n"]
    dil = []
    for psi in _evolve(H, psi0.astype(complex), times):
        dil.append([np.vdot(psi, _embed_one(n_op, s, N, d) @ psi).real for s in range(N)])
    dil = np.array(dil)
    # --- spin-1/2 XXZ with explicit fields, averaged over all 2^N configs
    sx = np.array([[0, 0.5], [0.5, 0]])
    sy = np.array([[0, -0.5j], [0.5j, 0]])
    sz = np.diag([0.5, -0.5])
    h2 = J * (np.kron(sx, sx) + np.kron(sy, sy)).real + V * np.kron(sz, sz)
    Hb = None
    for (i, j) in bonds:
        t = _embed_two(h2, i, j, N, 2)
        Hb = t if Hb is None else Hb + t
    Zs = [_embed_one(sz, s, N, 2) for s in range(N)]
    nloc = [_embed_one(np.diag([1.0, 0.0]), s, N, 2) for s in range(N)]
    phi0 = np.array([1.0])
    for s in range(N):
        phi0 = np.kron(phi0, np.eye(2)[neel[s]])
    avg = np.zeros((len(times), N))
    levels = [1.0 - 2.0 * a / (d_A - 1) for a in range(d_A)]
    for zs in itertools.product(levels, repeat=N):
        Hz = (Hb + sum(W * z * Z for z, Z in zip(zs, Zs))).toarray()
        lam, U = np.linalg.eigh(Hz)
        c0 = U.conj().T @ phi0
        for k, t in enumerate(times):
            phi = U @ (np.exp(-1j * t * lam) * c0)
            avg[k] += [np.vdot(phi, nloc[s] @ phi).real for s in range(N)]
    avg /= d_A ** N
    assert np.max(np.abs(dil - avg)) < 1e-12
