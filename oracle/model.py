"""Oracle: local Hilbert space, dilated bond Hamiltonian and Trotter gates.

Test infrastructure only (see package docstring).

Paper passages followed
    * Eq. (Hori): XXZ model with on-site fields h_i S^z_i.
    * "Set up for iPEPS", Initialization: one auxiliary spin per site with
      d_A = 2S+1 levels; |+> is the equal superposition of its levels.
    * Eq. (Hanc): the disorder enters as h * S^z_{ip} S^z_{ia}; the auxiliary
      S^z values are equally spaced in [-h, h] (d_A = 2: ±h; d_A = 3: h, 0, -h).

Readings (where the paper leaves the choice open)
    * spin operators are S = sigma/2 (paper says "Pauli spin operators");
    * the XY coefficient is J, the S^z S^z coefficient V (the paper's Delta),
      the field strength W (the paper's h);
    * local index s = p * d_A + a with p = 0 the occupied spin-up state;
      auxiliary level a carries z(a) = 1 - 2a/(d_A - 1) in [-1, 1];
    * each site's field is split over its four bonds, weight w = 1/4 per bond,
      inside the bond gate.

Pins (tests/test_oracle_model.py): gate unitarity, gate(τ)gate(-τ) = 1,
eigen-decomposition exponential equals scipy expm, and the dilation identity
(exact diagonalisation of the dilated cluster equals the explicit average
over all 2^N field configurations of the spin-1/2 cluster).
"""
import numpy as np
import scipy.linalg


def aux_levels(d_A):
    """z(a) for a = 0..d_A-1, equally spaced in [-1, 1] (Eq. Hanc text)."""
    if d_A == 1:
        return np.zeros(1)
    return np.array([1.0 - 2.0 * a / (d_A - 1) for a in range(d_A)])


def local_operators(d_A):
    """Operators on one site of dimension d = 2 d_A, index s = p*d_A + a.

    Returns dict with Sz, Sp (raising), Sm, Za (aux z), n (occupation),
    identity.  p = 0 is spin up = occupied (n = Sz + 1/2).
    """
    sz = np.diag([0.5, -0.5])
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])  # |up><down|
    ia = np.eye(d_A)
    za = np.diag(aux_levels(d_A))
    ops = {
        "Sz": np.kron(sz, ia),
        "Sp": np.kron(sp, ia),
        "Sm": np.kron(sp.T, ia),
        "Za": np.kron(np.eye(2), za),
        "I": np.eye(2 * d_A),
    }
    ops["n"] = ops["Sz"] + 0.5 * ops["I"]
    return ops


def bond_hamiltonian(J, V, W, w, d_A):
    """Two-site term h_b on (site i, site j), matrix index s_i*d + s_j.

    h_b = J (Sx Sx + Sy Sy) + V Sz Sz + w W (Sz Za (x) 1 + 1 (x) Sz Za),
    with Sx Sx + Sy Sy = (S+ S- + S- S+)/2.  Real symmetric.
    """
    o = local_operators(d_A)
    kron = np.kron
    h = 0.5 * J * (kron(o["Sp"], o["Sm"]) + kron(o["Sm"], o["Sp"]))
    h = h + V * kron(o["Sz"], o["Sz"])
    f = o["Sz"] @ o["Za"]
    h = h + w * W * (kron(f, o["I"]) + kron(o["I"], f))
    return h


def gate(h, tau):
    """G(tau) = exp(-i tau h) by scipy's matrix exponential."""
    return scipy.linalg.expm(-1j * tau * h)


# layer ids used by the Trotter schedule and by the per-layer test hooks
H_A, H_B, V_A, V_B = 0, 1, 2, 3


class Params:
    """Model + algorithm parameters of one job.

    layer_J / layer_V multiply J and V on the bonds of each layer; layer_w is
    the field weight w on each layer's bonds (default 1/4: every site has four
    bonds).  The hooks exist only to build exactly solvable limits in tests.
    """

    def __init__(self, D, chi, J=1.0, V=1.0, W=5.0, dt=0.05, d_A=2,
                 layer_J=(1, 1, 1, 1), layer_V=(1, 1, 1, 1),
                 layer_w=(0.25, 0.25, 0.25, 0.25)):
        self.D, self.chi, self.J, self.V, self.W, self.dt = D, chi, J, V, W, dt
        self.d_A = d_A
        self.d = 2 * d_A
        self.layer_J = tuple(float(x) for x in layer_J)
        self.layer_V = tuple(float(x) for x in layer_V)
        self.layer_w = tuple(float(x) for x in layer_w)

    def layer_hamiltonian(self, layer):
        return bond_hamiltonian(self.J * self.layer_J[layer],
                                self.V * self.layer_V[layer],
                                self.W, self.layer_w[layer], self.d_A)

    def layer_gate(self, layer, tau):
        return gate(self.layer_hamiltonian(layer), tau)
