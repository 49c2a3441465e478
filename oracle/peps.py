"""Oracle: 2x2-cell iPEPS, Néel ⊗ |+> initial state, plain simple update.

Test infrastructure only (see package docstring).

Paper passages followed
    * Initialization: Néel physical state ⊗ |+> auxiliary state, a product
      state, i.e. an iPEPS of bond dimension D = 1 on a checkerboard cell
      (Fig. 1 caption).
    * Quench: real-time evolution e^{-iHt} by the simple update of the
      dilated Hamiltonian Eq. (Hanc), Trotter steps δt (appendix).
    * Local truncation error: sum of squared discarded weights for one site.

Data layout of one state (a plain dict, see ``new_state``)
    gam[(x, y)]   complex (d, D, D, D, D), legs (s, up, left, down, right)
    lam_h[(x, y)] real (D,), bond between (x, y).right and (x+1, y).left
    lam_v[(x, y)] real (D,), bond between (x, y).down and (x, y+1).up
    eps[(x, y)]   accumulated truncation error of the site
Coordinates are taken mod 2; y grows downwards.  Sites with x+y even are
the A (initially occupied) sublattice.

Readings (where the paper leaves the choice open): the 2x2 cell with
checkerboard layers, a symmetric second-order Trotter step H_A/2 H_B/2 V_A/2
V_B V_A/2 H_B/2 H_A/2 (layers never merged across steps), the truncation
rule ``trunc_rule``, lambda normalised to unit 2-norm, pseudo-inverse cutoff
1e-14 relative, site tensors normalised to max |.| = 1 after each update,
and the per-update error sum_{k>g} s_k^2 / sum_k s_k^2 added to both end
sites.

The bond update here is the *plain* form: the full SVD of the
(d D^3) x (d D^3) two-site matrix.  Any reduced (QR) form gives the same
singular values and truncated state up to gauge.

Pins: tests/test_oracle_peps.py (zero hopping keeps the state a product,
D = 1 limit, dimer closed form, 1D XX chain Bessel law, symmetries,
particle-number conservation, checkerboard symmetry, short-time Taylor
coefficients).
"""
import numpy as np

from .model import H_A, H_B, V_A, V_B

SITES = [(0, 0), (1, 0), (0, 1), (1, 1)]
SV_ZERO_REL = 1e-12      # singular values at or below this * s_1 are zeros
MULTIPLET_REL = 1e-10    # relative gap below which two values are one multiplet
LAMBDA_INV_REL = 1e-14   # pseudo-inverse cutoff for 1/lambda

# Trotter layers: horizontal (H) bonds are named by their left site,
# vertical (V) bonds by their upper site; A = that site is on sublattice A.
LAYER_BONDS = {
    H_A: [(0, 0), (1, 1)],
    H_B: [(1, 0), (0, 1)],
    V_A: [(0, 0), (1, 1)],
    V_B: [(1, 0), (0, 1)],
}
# one second-order step: (layer, fraction of dt)
TROTTER_SEQUENCE = [(H_A, 0.5), (H_B, 0.5), (V_A, 0.5), (V_B, 1.0),
                    (V_A, 0.5), (H_B, 0.5), (H_A, 0.5)]


def m2(x, y):
    return (x % 2, y % 2)


def is_A(site):
    return (site[0] + site[1]) % 2 == 0


def trunc_rule(s, K):
    """Number g of singular values kept out of the sorted list s, at most K.

    Values <= 1e-12 s_1 count as zeros and are never kept; when values are
    dropped, the cut is moved down so that it never separates two values
    whose gap is <= 1e-10 of the larger one plus 1e-12 s_1 (a multiplet is
    kept or dropped whole; the absolute part makes the decision independent
    of rounding-level splittings of small degenerate values).
    """
    s = np.asarray(s, dtype=float)
    if s.size == 0 or s[0] <= 0.0:
        return 0
    r = int(np.sum(s > SV_ZERO_REL * s[0]))
    g = min(K, r)
    if g < r:
        while g > 1 and s[g - 1] - s[g] <= MULTIPLET_REL * s[g - 1] + SV_ZERO_REL * s[0]:
            g -= 1
    return g


def new_state(params):
    """Néel ⊗ |+> as a D = 1 iPEPS embedded in bond dimension D."""
    D, d, d_A = params.D, params.d, params.d_A
    st = {"gam": {}, "lam_h": {}, "lam_v": {}, "eps": {}}
    for site in SITES:
        g = np.zeros((d, D, D, D, D), dtype=complex)
        p = 0 if is_A(site) else 1          # A: spin up (occupied)
        for a in range(d_A):
            g[p * d_A + a, 0, 0, 0, 0] = 1.0 / np.sqrt(d_A)
        st["gam"][site] = g
        lam = np.zeros(D)
        lam[0] = 1.0
        st["lam_h"][site] = lam.copy()
        st["lam_v"][site] = lam.copy()
        st["eps"][site] = 0.0
    return st


def copy_state(st):
    return {k: {s: (v.copy() if isinstance(v, np.ndarray) else v)
                for s, v in st[k].items()} for k in st}


def _inv(lam):
    out = np.zeros_like(lam)
    cut = LAMBDA_INV_REL * np.max(lam) if lam.size else 0.0
    mask = lam > cut
    out[mask] = 1.0 / lam[mask]
    return out


def _split(theta_mat, D):
    """SVD + truncation of the two-site matrix; returns U, s_kept, Vh, g, eps."""
    U, s, Vh = np.linalg.svd(theta_mat, full_matrices=False)
    g = trunc_rule(s, D)
    tot = float(np.sum(s ** 2))
    eps = float(np.sum(s[g:] ** 2)) / tot if tot > 0 else 0.0
    lam = np.zeros(D)
    if g > 0:
        lam[:g] = s[:g] / np.linalg.norm(s[:g])
    return U, lam, Vh, g, eps


def _gate4(G, d):
    return G.reshape(d, d, d, d)  # [s_i', s_j', s_i, s_j]


def update_horizontal(st, site, G, D):
    """Simple update of the bond (x,y).right -- (x+1,y).left with gate G."""
    x, y = site
    i, j = m2(x, y), m2(x + 1, y)
    gi, gj = st["gam"][i], st["gam"][j]
    d = gi.shape[0]
    lu_i, ll_i, ld_i = st["lam_v"][m2(x, y - 1)], st["lam_h"][m2(x - 1, y)], st["lam_v"][i]
    lu_j, ld_j, lr_j = st["lam_v"][m2(x + 1, y - 1)], st["lam_v"][j], st["lam_h"][j]
    lb = st["lam_h"][i]
    Mi = np.einsum("sulde,u,l,d->sulde", gi, lu_i, ll_i, ld_i)
    Mj = np.einsum("tvewx,v,w,x->tvewx", gj, lu_j, ld_j, lr_j)
    theta = np.einsum("sulde,e,tvewx->suldtvwx", Mi, lb, Mj)
    theta = np.einsum("abst,suldtvwx->auldbvwx", _gate4(G, d), theta)
    U, lam, Vh, g, eps = _split(theta.reshape(d * D ** 3, d * D ** 3), D)
    ni = np.zeros((d, D, D, D, D), dtype=complex)
    nj = np.zeros((d, D, D, D, D), dtype=complex)
    ni[..., :g] = U[:, :g].reshape(d, D, D, D, g)
    ni = np.einsum("sulde,u,l,d->sulde", ni, _inv(lu_i), _inv(ll_i), _inv(ld_i))
    vj = Vh[:g, :].reshape(g, d, D, D, D)            # [k, t, v, w, x]
    nj[:, :, :g, :, :] = np.transpose(vj, (1, 2, 0, 3, 4))
    nj = np.einsum("tvewx,v,w,x->tvewx", nj, _inv(lu_j), _inv(ld_j), _inv(lr_j))
    return i, j, ni / np.max(np.abs(ni)), nj / np.max(np.abs(nj)), lam, eps


def update_vertical(st, site, G, D):
    """Simple update of the bond (x,y).down -- (x,y+1).up with gate G."""
    x, y = site
    i, j = m2(x, y), m2(x, y + 1)
    gi, gj = st["gam"][i], st["gam"][j]
    d = gi.shape[0]
    lu_i, ll_i, lr_i = st["lam_v"][m2(x, y - 1)], st["lam_h"][m2(x - 1, y)], st["lam_h"][i]
    ll_j, ld_j, lr_j = st["lam_h"][m2(x - 1, y + 1)], st["lam_v"][j], st["lam_h"][j]
    lb = st["lam_v"][i]
    Mi = np.einsum("sulkr,u,l,r->sulkr", gi, lu_i, ll_i, lr_i)
    Mj = np.einsum("tkmwx,m,w,x->tkmwx", gj, ll_j, ld_j, lr_j)
    theta = np.einsum("sulkr,k,tkmwx->sulrtmwx", Mi, lb, Mj)
    theta = np.einsum("abst,sulrtmwx->aulrbmwx", _gate4(G, d), theta)
    U, lam, Vh, g, eps = _split(theta.reshape(d * D ** 3, d * D ** 3), D)
    ni = np.zeros((d, D, D, D, D), dtype=complex)
    nj = np.zeros((d, D, D, D, D), dtype=complex)
    ui = U[:, :g].reshape(d, D, D, D, g)               # [s, u, l, r, k]
    ni[:, :, :, :g, :] = np.transpose(ui, (0, 1, 2, 4, 3))
    ni = np.einsum("sulkr,u,l,r->sulkr", ni, _inv(lu_i), _inv(ll_i), _inv(lr_i))
    vj = Vh[:g, :].reshape(g, d, D, D, D)              # [k, t, m, w, x]
    nj[:, :g, :, :, :] = np.transpose(vj, (1, 0, 2, 3, 4))
    nj = np.einsum("tkmwx,m,w,x->tkmwx", nj, _inv(ll_j), _inv(ld_j), _inv(lr_j))
    return i, j, ni / np.max(np.abs(ni)), nj / np.max(np.abs(nj)), lam, eps


def apply_layer(st, params, layer, tau):
    """Apply the gates of one layer; both bonds see the pre-layer state."""
    G = params.layer_gate(layer, tau)
    horizontal = layer in (H_A, H_B)
    results = []
    for site in LAYER_BONDS[layer]:
        fn = update_horizontal if horizontal else update_vertical
        results.append((site, fn(st, site, G, params.D)))
    for site, (i, j, ni, nj, lam, eps) in results:
        st["gam"][i], st["gam"][j] = ni, nj
        (st["lam_h"] if horizontal else st["lam_v"])[m2(*site)] = lam
        st["eps"][i] += eps
        st["eps"][j] += eps


def trotter_step(st, params):
    """One symmetric second-order Trotter step (7 layers, 14 bond updates)."""
    for layer, frac in TROTTER_SEQUENCE:
        apply_layer(st, params, layer, frac * params.dt)


def bond_spectra(st):
    """The 8 bond weight vectors in the order h(0,0) h(1,0) h(0,1) h(1,1),
    v(0,0) v(1,0) v(0,1) v(1,1)."""
    return np.array([st["lam_h"][s] for s in SITES] + [st["lam_v"][s] for s in SITES])
