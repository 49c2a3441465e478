"""Oracle: double-layer tensors, directional CTMRG, one-site readout.

Test infrastructure only (see package docstring).

Paper passages followed
    * Readout: on-site expectation values at the physical site with the
      auxiliary spin traced out, from an instance of CTMRG; Rényi entropies
      from the same environment.
    * Appendix: CTMRG contracts the whole infinite lattice except one site;
      environment bond dimension chi >= D^2, converged.
    * Results (interacting case): particle number on the two sublattices and
      the imbalance, their difference.

The paper gives no CTMRG details; this module takes the common directional
CTMRG for a 2x2 unit cell with half-system projectors (these readings fill
what the paper leaves open):
    * environment of every site: corners C1..C4 (top-left, top-right,
      bottom-right, bottom-left) and edges T1..T4 (up, right, down, left);
      C_k has legs [prev, next] and T_k legs [prev, q, next], going clockwise
      around the ring C1 T1 C2 T2 C3 T3 C4 T4, q being the double-layer leg;
    * cold start: every C and T is the neighbouring double-layer tensor with
      its outward legs closed by the boundary vector (identity for a PEPS),
      embedded in chi;
    * a left move absorbs column x into the left environment of column x+1,
      for x = 0 then 1; the projectors of the cut between rows y and y+1 come
      from the 2x2 block of sites (x,y) (x+1,y) (x+1,y+1) (x,y+1): with the
      four enlarged corners UL UR DR DL, F = UL UR, G = DR DL, N = G F = U S V^H
      truncated to g <= chi values (``trunc_rule``), P_low = F V S^{-1/2}
      contracts the lower tensors, P_up = S^{-1/2} U^H G the upper ones;
    * the right, up and down moves are the left move on the lattice rotated
      by 180, 90 and 270 degrees; one iteration is left, right, up, down;
    * every new C and T is divided by its Frobenius norm;
    * convergence: singular values of all 16 corners normalised to unit
      2-norm; delta = largest 2-norm change over one iteration.

Pins: tests/test_oracle_ctmrg.py (Onsager magnetisation of the 2D Ising
model through the same CTMRG, product-state exactness at any chi, cold-start
invariants, basis-independence of the spectra).
"""
import numpy as np

from .peps import SITES, m2, trunc_rule


# ---------------------------------------------------------------- double layer
def absorb_sqrt_lambda(st, site):
    """A = Gamma with sqrt(lambda) on each of its four legs."""
    x, y = site
    lu = np.sqrt(st["lam_v"][m2(x, y - 1)])
    ll = np.sqrt(st["lam_h"][m2(x - 1, y)])
    ld = np.sqrt(st["lam_v"][m2(x, y)])
    lr = np.sqrt(st["lam_h"][m2(x, y)])
    return np.einsum("suldr,u,l,d,r->suldr", st["gam"][m2(x, y)], lu, ll, ld, lr)


def double_layer(A):
    """a[(u u'),(l l'),(d d'),(r r')] = sum_s A[s,u,l,d,r] conj(A[s,u',l',d',r'])."""
    D = A.shape[1]
    a = np.einsum("suldr,sULDR->uUlLdDrR", A, A.conj())
    return a.reshape(D * D, D * D, D * D, D * D)


def identity_boundary(D):
    return np.eye(D).reshape(D * D).astype(complex)


# ---------------------------------------------------------------- lattice frames
def rotate(lat):
    """Rotate a 2x2-cell lattice (site tensors + environments) by one quarter
    turn so that the physical 'up' direction becomes the frame's 'left'.

    frame leg order (U, L, D, R) = physical (right, up, left, down);
    frame corner/edge k = physical corner/edge k+1; frame site (X, Y) =
    physical (y, -x).
    """
    a_new, env_new = {}, {}
    for (x, y), a in lat["a"].items():
        X, Y = m2(y, -x)
        a_new[(X, Y)] = np.transpose(a, (3, 0, 1, 2))
        if lat.get("env") is not None:
            e = lat["env"][(x, y)]
            env_new[(X, Y)] = {"C": [e["C"][(k + 1) % 4] for k in range(4)],
                               "T": [e["T"][(k + 1) % 4] for k in range(4)]}
    return {"a": a_new, "env": env_new if lat.get("env") is not None else None}


def rotate_n(lat, n):
    for _ in range(n % 4):
        lat = rotate(lat)
    return lat


# ---------------------------------------------------------------- environment
def _embed(t, shape):
    out = np.zeros(shape, dtype=complex)
    out[tuple(slice(0, s) for s in t.shape)] = t
    return out


def init_environment(a, chi, bvec):
    """Cold start: neighbouring tensors with outward legs closed by bvec."""
    q = next(iter(a.values())).shape[0]
    if chi < q:
        raise ValueError("chi must be >= the double-layer leg dimension")
    b = bvec
    env = {}
    for (x, y) in SITES:
        C1 = np.einsum("uldr,u,l->dr", a[m2(x - 1, y - 1)], b, b)
        T1 = np.einsum("uldr,u->ldr", a[m2(x, y - 1)], b)
        C2 = np.einsum("uldr,u,r->ld", a[m2(x + 1, y - 1)], b, b)
        T2 = np.einsum("uldr,r->uld", a[m2(x + 1, y)], b)
        C3 = np.einsum("uldr,d,r->ul", a[m2(x + 1, y + 1)], b, b)
        T3 = np.einsum("uldr,d->rul", a[m2(x, y + 1)], b)
        C4 = np.einsum("uldr,l,d->ru", a[m2(x - 1, y + 1)], b, b)
        T4 = np.einsum("uldr,l->dru", a[m2(x - 1, y)], b)
        env[(x, y)] = {
            "C": [_embed(c, (chi, chi)) for c in (C1, C2, C3, C4)],
            "T": [_embed(t, (chi, q, chi)) for t in (T1, T2, T3, T4)],
        }
    return env


def enlarged_corner(C, Tprev, Tnext, arot):
    """Top-left enlarged corner as a matrix [prev, next] of size (chi q)^2.

    prev = (Tprev.prev, a.down), next = (Tnext.next, a.right), for the site
    tensor rotated so that this corner is its top-left one.
    """
    chi, q = C.shape[0], arot.shape[0]
    X1 = np.einsum("ab,buc->auc", C, Tnext, optimize=True)
    X2 = np.einsum("dla,auc->dluc", Tprev, X1, optimize=True)
    E = np.einsum("dluc,uler->decr", X2, arot, optimize=True)
    return E.reshape(chi * q, chi * q)


def _rot_a(a, k):
    for _ in range(k % 4):
        a = np.transpose(a, (3, 0, 1, 2))
    return a


def block_corners(lat, X, Y):
    """UL, UR, DR, DL enlarged corners of the 2x2 block with top-left (X, Y)."""
    env, a = lat["env"], lat["a"]
    out = []
    for k, site in enumerate([m2(X, Y), m2(X + 1, Y), m2(X + 1, Y + 1), m2(X, Y + 1)]):
        e = env[site]
        out.append(enlarged_corner(e["C"][k], e["T"][(k - 1) % 4], e["T"][k],
                                   _rot_a(a[site], k)))
    return out


def projectors(UL, UR, DR, DL, chi):
    """Half-system projectors of the left cut of one 2x2 block."""
    F = UL @ UR
    G = DR @ DL
    N = G @ F
    U, S, Vh = np.linalg.svd(N)
    g = trunc_rule(S, chi)
    n = N.shape[0]
    P_low = np.zeros((n, chi), dtype=complex)
    P_up = np.zeros((chi, n), dtype=complex)
    if g > 0:
        w = 1.0 / np.sqrt(S[:g])
        P_low[:, :g] = (F @ Vh[:g].conj().T) * w[None, :]
        P_up[:g, :] = w[:, None] * (U[:, :g].conj().T @ G)
    return P_low, P_up, S, g


def left_move(lat, chi):
    """Absorb column 0 into column 1, then column 1 into column 0."""
    env, a = lat["env"], lat["a"]
    q = next(iter(a.values())).shape[0]
    for X in (0, 1):
        P = {}
        for Y in (0, 1):
            UL, UR, DR, DL = block_corners(lat, X, Y)
            P[Y] = projectors(UL, UR, DR, DL, chi)[:2]
        new = {}
        for Y in (0, 1):
            P_low, P_up = P[Y]
            P_low_prev = P[(Y - 1) % 2][0]
            # C1 of (X+1, Y+1): C1(X, Y+1) T1(X, Y+1), down leg cut by P_up(Y)
            e = env[m2(X, Y + 1)]
            C1T1 = np.einsum("ab,bqc->aqc", e["C"][0], e["T"][0]).reshape(chi * q, chi)
            new[("C1", m2(X + 1, Y + 1))] = P_up @ C1T1
            # C4 of (X+1, Y): C4(X, Y) T3(X, Y), up leg cut by P_low(Y)
            e = env[m2(X, Y)]
            T3C4 = np.einsum("pqc,cn->pnq", e["T"][2], e["C"][3]).reshape(chi, chi * q)
            new[("C4", m2(X + 1, Y))] = T3C4 @ P_low
            # T4 of (X+1, Y): P_up(Y) [T4(X,Y) a(X,Y)] P_low(Y-1)
            Pu3 = P_up.reshape(chi, chi, q)
            Pl3 = P_low_prev.reshape(chi, q, chi)
            W1 = np.einsum("ctd,tln->cdln", Pu3, e["T"][3], optimize=True)
            W2 = np.einsum("cdln,uldr->cnur", W1, a[m2(X, Y)], optimize=True)
            new[("T4", m2(X + 1, Y))] = np.einsum("cnur,nue->cre", W2, Pl3, optimize=True)
        for (name, site), t in new.items():
            nrm = np.linalg.norm(t)
            t = t / nrm if nrm > 0 else t
            if name == "C1":
                env[site]["C"][0] = t
            elif name == "C4":
                env[site]["C"][3] = t
            else:
                env[site]["T"][3] = t
    return lat


# physical rotation used by each move: left, right, up, down
MOVES = (0, 2, 1, 3)


def ctmrg_iteration(lat, chi):
    for f in MOVES:
        r = rotate_n(lat, f)
        left_move(r, chi)
        lat = rotate_n(r, 4 - f)
    return lat


def corner_spectra(env, chi):
    """(16, chi) array: normalised singular values of C1..C4 of every site."""
    out = np.zeros((16, chi))
    i = 0
    for site in SITES:
        for k in range(4):
            s = np.linalg.svd(env[site]["C"][k], compute_uv=False)
            nrm = np.linalg.norm(s)
            out[i, :s.size] = s / nrm if nrm > 0 else s
            i += 1
    return out


def ctmrg(a, chi, env=None, bvec=None, max_iter=10, tol=None):
    """Run CTMRG on site tensors a[(x,y)] (legs u,l,d,r).

    tol None: exactly max_iter iterations.  Otherwise stop after the first
    iteration with delta < tol (or at max_iter).  Returns (env, iters, delta).
    """
    if env is None:
        if bvec is None:
            q = next(iter(a.values())).shape[0]
            bvec = identity_boundary(int(round(np.sqrt(q))))
        env = init_environment(a, chi, bvec)
    lat = {"a": a, "env": env}
    prev = corner_spectra(env, chi)
    delta, it = np.inf, 0
    for it in range(1, max_iter + 1):
        lat = ctmrg_iteration(lat, chi)
        cur = corner_spectra(lat["env"], chi)
        delta = float(np.max(np.linalg.norm(cur - prev, axis=1)))
        prev = cur
        if tol is not None and delta < tol:
            break
    return lat["env"], it, delta


# ---------------------------------------------------------------- readout
def site_environment(e):
    """Ring contraction of C1 T1 C2 T2 C3 T3 C4 T4 -> E[q_u, q_l, q_d, q_r]."""
    C1, C2, C3, C4 = e["C"]
    T1, T2, T3, T4 = e["T"]
    upper = np.einsum("ab,buc,cd->aud", C1, T1, C2, optimize=True)   # [C1.prev, q_u, C2.next]
    lower = np.einsum("ef,fvg,gh->ehv", C3, T3, C4, optimize=True)   # [C3.prev, C4.next, q_d]
    UR = np.einsum("aud,dre->aure", upper, T2, optimize=True)
    LL = np.einsum("ehv,hla->evla", lower, T4, optimize=True)
    E = np.einsum("aure,evla->ulvr", UR, LL, optimize=True)
    return E


def reduced_density_matrix(E, A):
    """rho[s, s'] = contraction of E with A_s (x) conj(A_s'), trace normalised."""
    D = A.shape[1]
    E8 = E.reshape(D, D, D, D, D, D, D, D)
    half = np.einsum("uUlLdDrR,suldr->sULDR", E8, A, optimize=True)
    rho = np.einsum("sULDR,tULDR->st", half, A.conj(), optimize=True)
    return rho / np.trace(rho)


def renyi(rp):
    """Renyi entropies S_1 = -Tr r ln r and S_1/2 = 2 ln Tr sqrt(r) of a
    Hermitian unit-trace matrix r (section Results: entropies of the one-site
    reduced density matrix, orders 1 and 1/2; natural log, maximum ln d_p)."""
    lam = np.clip(np.linalg.eigvalsh(0.5 * (rp + rp.conj().T)), 0.0, None)
    nz = lam[lam > 0]
    return float(-(nz * np.log(nz)).sum()), float(2.0 * np.log(np.sqrt(lam).sum()))


def observe(st, env, d_A):
    """Occupations n(x,y) (aux traced), imbalance, sum of n, max |rho_p[up,dn]|,
    Renyi S_1 and S_1/2 of each physical one-site matrix rho_p."""
    n, s1, sh = {}, {}, {}
    offd = 0.0
    for site in SITES:
        A = absorb_sqrt_lambda(st, site)
        rho = reduced_density_matrix(site_environment(env[site]), A)
        rp = np.einsum("paqa->pq", rho.reshape(2, d_A, 2, d_A))
        n[site] = float(rp[0, 0].real)
        offd = max(offd, abs(rp[0, 1]))
        s1[site], sh[site] = renyi(rp)
    imb = 0.5 * (n[(0, 0)] + n[(1, 1)] - n[(1, 0)] - n[(0, 1)])
    return {"n": np.array([n[s] for s in SITES]), "imbalance": imb,
            "sum_n": float(sum(n.values())), "max_offdiag": float(offd),
            "renyi1": np.array([s1[s] for s in SITES]),
            "renyi_half": np.array([sh[s] for s in SITES])}


def double_layers(st):
    return {site: double_layer(absorb_sqrt_lambda(st, site)) for site in SITES}
