// Simple update on the device (FP64, complex): Trotter gates and bond updates.
//
// A bond update of sites i -- j (bond weights lambda_b):
//   M_X[(outer legs), (s, bond)] = Gamma_X * outer lambdas          (D^3 x dD)
//   M_X = Q_X R_X                         Householder QR, R_X is r x dD
//   Theta'[(k_i, s_i'), (s_j', k_j)] = sum_b lambda_b sum_{s_i s_j}
//        G[(s_i' s_j'), (s_i s_j)] R_i[k_i, (s_i, b)] R_j[k_j, (s_j, b)]
//   Theta' = U S V^H                      one-sided (Hestenes) Jacobi, FP64, on
//                                         R^H of a column-pivoted QR of Theta'
//   keep g <= D values (zeros <= 1e-12 s_1 dropped, multiplets -- gaps <=
//   1e-10 s_g + 1e-12 s_1 -- kept whole)
//   Gamma_i' = Q_i U_g / outer lambdas,  Gamma_j' = Q_j conj(V_g) / outer lambdas
//   lambda_b' = s_g / |s_g|,  eps += sum_{k >= g} s_k^2 / sum_k s_k^2 on i and j
//   Gamma' /= max |Gamma'|
// The reduced matrix has the same singular values and truncated state (up to
// gauge) as the full (d D^3) x (d D^3) two-site matrix.  One workgroup per
// bond; the two bonds of a layer touch disjoint sites and run together.
#include "su.h"

#include <cmath>

namespace ipeps {

// ------------------------------------------------------------------ gates
struct GateParams {
    int d_A;
    double J[4], V[4], w[4];
    double W, dt;
};

// h_b conserves both auxiliary labels and the number of up spins, so
// exp(-i tau h_b) splits into blocks per (a_i, a_j): phases on |up up> and
// |dn dn>, and a 2 x 2 unitary on {|up dn>, |dn up>} with the closed form
// exp(-i tau (m0 + m.sigma)) = e^{-i tau m0} (cos(tau|m|) - i sin(tau|m|) m.sigma/|m|).
__global__ void k_build_gates(GateParams gp, cplx* gates) {
    const int layer = blockIdx.x >> 1, which = blockIdx.x & 1;
    const int dA = gp.d_A, d = 2 * dA, dd = d * d;
    const double Jl = gp.J[layer], Vl = gp.V[layer], wW = gp.w[layer] * gp.W;
    const double tau = which ? gp.dt : 0.5 * gp.dt;
    cplx* G = gates + (long)blockIdx.x * dd * dd;
    for (long e = threadIdx.x; e < (long)dd * dd; e += blockDim.x) G[e] = cmake(0, 0);
    __syncthreads();
    for (int blk = threadIdx.x; blk < dA * dA; blk += blockDim.x) {
        const int ai = blk / dA, aj = blk % dA;
        const double zi = dA > 1 ? 1.0 - 2.0 * ai / (dA - 1) : 0.0;
        const double zj = dA > 1 ? 1.0 - 2.0 * aj / (dA - 1) : 0.0;
        auto idx = [&](int pi, int pj) { return (pi * dA + ai) * d + (pj * dA + aj); };
        auto phase = [&](double E) { return cmake(cos(tau * E), -sin(tau * E)); };
        // S^z = +1/2 for p = 0 (up), -1/2 for p = 1
        const double e00 = 0.25 * Vl + 0.5 * wW * (zi + zj);
        const double e11 = 0.25 * Vl - 0.5 * wW * (zi + zj);
        const double e01 = -0.25 * Vl + 0.5 * wW * (zi - zj);
        const double e10 = -0.25 * Vl - 0.5 * wW * (zi - zj);
        G[(long)idx(0, 0) * dd + idx(0, 0)] = phase(e00);
        G[(long)idx(1, 1) * dd + idx(1, 1)] = phase(e11);
        const double m0 = 0.5 * (e01 + e10), mz = 0.5 * (e01 - e10), mx = 0.5 * Jl;
        const double mm = sqrt(mz * mz + mx * mx);
        const double c = cos(tau * mm), sn = mm > 0 ? sin(tau * mm) / mm : tau;
        const cplx ph = phase(m0);
        const int u = idx(0, 1), v = idx(1, 0);
        G[(long)u * dd + u] = cmul(ph, cmake(c, -sn * mz));
        G[(long)v * dd + v] = cmul(ph, cmake(c, sn * mz));
        G[(long)u * dd + v] = cmul(ph, cmake(0, -sn * mx));
        G[(long)v * dd + u] = cmul(ph, cmake(0, -sn * mx));
    }
}

void build_gates(hipStream_t s, const ipeps_config& cfg, cplx* gates) {
    GateParams gp;
    gp.d_A = cfg.d_A;
    for (int l = 0; l < 4; ++l) {
        gp.J[l] = cfg.J * cfg.layer_J[l];
        gp.V[l] = cfg.V * cfg.layer_V[l];
        gp.w[l] = cfg.layer_w[l];
    }
    gp.W = cfg.W;
    gp.dt = cfg.dt;
    hipLaunchKernelGGL(k_build_gates, dim3(8), dim3(256), 0, s, gp, gates);
    HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ bond update
struct SuDims {
    int D, d, Dc, nb, r, m;  // Dc = D^3, nb = d D, r = min(Dc, nb), m = d r
};

__host__ __device__ inline SuDims su_dims(int D, int d) {
    SuDims s;
    s.D = D;
    s.d = d;
    s.Dc = D * D * D;
    s.nb = d * D;
    s.r = s.Dc < s.nb ? s.Dc : s.nb;
    s.m = d * s.r;
    return s;
}

struct SuScratch {
    cplx *Mi, *Mj, *taui, *tauj, *Th, *Ac, *U, *B, *Xi, *Xj;
    double* sig;
};

__host__ __device__ inline size_t su_layout(const SuDims& s, char* base, SuScratch* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const size_t cm = (size_t)s.Dc * s.nb * sizeof(cplx);
    SuScratch t;
    t.Mi = (cplx*)take(cm);
    t.Mj = (cplx*)take(cm);
    t.taui = (cplx*)take(s.nb * sizeof(cplx));
    t.tauj = (cplx*)take(s.nb * sizeof(cplx));
    t.Th = (cplx*)take((size_t)s.m * s.m * sizeof(cplx));
    t.Ac = (cplx*)take((size_t)s.m * s.m * sizeof(cplx));
    t.U = (cplx*)take((size_t)s.m * s.D * sizeof(cplx));
    t.B = (cplx*)take((size_t)s.m * s.D * sizeof(cplx));
    t.Xi = (cplx*)take(cm);
    t.Xj = (cplx*)take(cm);
    t.sig = (double*)take((size_t)s.m * sizeof(double));
    if (out) *out = t;
    return off;
}

size_t su_scratch_bytes(int D, int d) { return 2 * su_layout(su_dims(D, d), nullptr, nullptr); }

// Leg values (u, l, d, r) of a site tensor from the outer-leg row index and
// the bond index.
__device__ inline long gam_offset(int D, int bond_leg, int row, int s, int b) {
    int o[3] = {row / (D * D), (row / D) % D, row % D};
    int leg[5];
    int k = 0;
    for (int p = 1; p <= 4; ++p) leg[p] = (p == bond_leg) ? b : o[k++];
    const long D2 = (long)D * D;
    return (long)s * D2 * D2 + (long)leg[1] * D2 * D + (long)leg[2] * D2 + (long)leg[3] * D +
           leg[4];
}

// Householder QR of the column-major Dc x nb matrix M in place (LAPACK
// zgeqr2 conventions: R in the upper triangle, v_j below the diagonal with
// v_j[j] = 1 implicit, H_j = I - tau_j v_j v_j^H).
__device__ void householder_qr(int Dc, int nb, int r, cplx* M, cplx* tau, double* red,
                               cplx* bcast) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = 0; j < r; ++j) {
        cplx* col = M + (long)j * Dc;
        double s = 0;
        for (int i = j + 1 + threadIdx.x; i < Dc; i += blockDim.x) s += cabs2(col[i]);
        s = block_sum(s, red);
        if (threadIdx.x == 0) {
            const cplx alpha = col[j];
            cplx t = cmake(0, 0), scale = cmake(0, 0);
            if (!(s == 0.0 && alpha.im == 0.0)) {
                const double nrm = sqrt(cabs2(alpha) + s);
                const double beta = alpha.re >= 0 ? -nrm : nrm;
                t = cmake((beta - alpha.re) / beta, -alpha.im / beta);
                const cplx den = cmake(alpha.re - beta, alpha.im);  // 1 / (alpha - beta)
                const double dn = cabs2(den);
                scale = cmake(den.re / dn, -den.im / dn);
                col[j] = cmake(beta, 0.0);
            }
            tau[j] = t;
            bcast[0] = scale;
        }
        __syncthreads();
        const cplx sc = bcast[0];
        const cplx tj = tau[j];
        if (tj.re != 0.0 || tj.im != 0.0)
            for (int i = j + 1 + threadIdx.x; i < Dc; i += blockDim.x) col[i] = cmul(col[i], sc);
        __syncthreads();
        if (tj.re != 0.0 || tj.im != 0.0) {
            // a_c -= conj(tau) v (v^H a_c) for the trailing columns
            for (int c = j + 1 + wave; c < nb; c += nw) {
                cplx* ac = M + (long)c * Dc;
                cplx w = cmake(0, 0);
                for (int i = j + lane; i < Dc; i += 64) {
                    const cplx v = (i == j) ? cmake(1, 0) : col[i];
                    w = cadd(w, cdotc(v, ac[i]));
                }
                w.re = wave_sum(w.re);
                w.im = wave_sum(w.im);
                const cplx f = cmul(cconj(tj), w);
                for (int i = j + lane; i < Dc; i += 64) {
                    const cplx v = (i == j) ? cmake(1, 0) : col[i];
                    ac[i] = csub(ac[i], cmul(f, v));
                }
            }
        }
        __syncthreads();
    }
}

// X (Dc x ncols, column-major) <- Q X with Q = H_0 H_1 ... H_{r-1}.
__device__ void householder_apply_q(int Dc, int r, int ncols, const cplx* M, const cplx* tau,
                                    cplx* X) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = r - 1; j >= 0; --j) {
        const cplx tj = tau[j];
        if (tj.re == 0.0 && tj.im == 0.0) continue;
        const cplx* v = M + (long)j * Dc;
        for (int c = wave; c < ncols; c += nw) {
            cplx* xc = X + (long)c * Dc;
            cplx w = cmake(0, 0);
            for (int i = j + lane; i < Dc; i += 64) {
                const cplx vi = (i == j) ? cmake(1, 0) : v[i];
                w = cadd(w, cdotc(vi, xc[i]));
            }
            w.re = wave_sum(w.re);
            w.im = wave_sum(w.im);
            const cplx f = cmul(tj, w);
            for (int i = j + lane; i < Dc; i += 64) {
                const cplx vi = (i == j) ? cmake(1, 0) : v[i];
                xc[i] = csub(xc[i], cmul(f, vi));
            }
        }
        __syncthreads();
    }
}

// One-sided complex Jacobi on the columns of the m x n column-major A; one
// group of 16 lanes per column pair (DPP sums inside the group).
__device__ void complex_jacobi(int m, int n, cplx* A, int* flag, double* red) {
    const int g16 = threadIdx.x & 15, group = threadIdx.x >> 4, ngroups = blockDim.x >> 4;
    const int ne = n + (n & 1), npair = ne / 2;
    // A pair is rotated unless orthogonal to 1e-15 relative; the sweeps end
    // once no rotation angle exceeds 1e-14.  The angle, not the inner
    // product, decides convergence: for two columns whose norms differ by a
    // relative gap delta, an inner product left at tol |a_p| |a_q| mixes
    // their directions by ~tol / delta, which enters the truncated state
    // when the pair straddles the cut; well separated pairs still rotate by
    // rounding-level angles, which do not count.
    const double tol = 1e-15, tmin = 1e-14;
    // columns below 1e-14 |A|_F are rounding noise and are left alone
    double fro = 0.0;
    for (long e = threadIdx.x; e < (long)m * n; e += blockDim.x) fro += cabs2(A[e]);
    fro = block_sum(fro, red);
    const double small2 = 1e-28 * fro;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int rr = 0; rr < ne - 1; ++rr) {
            for (int k = group; k < npair; k += ngroups) {
                int p, q;
                if (k == 0) {
                    p = rr;
                    q = ne - 1;
                } else {
                    p = (rr + k) % (ne - 1);
                    q = (rr - k + ne - 1) % (ne - 1);
                }
                if (p > q) {
                    int t = p;
                    p = q;
                    q = t;
                }
                if (q >= n) continue;
                cplx* ap = A + (long)p * m;
                cplx* aq = A + (long)q * m;
                double al = 0, be = 0, gr = 0, gi = 0;
                for (int i = g16; i < m; i += 16) {
                    const cplx x = ap[i], y = aq[i];
                    al += cabs2(x);
                    be += cabs2(y);
                    const cplx g = cdotc(x, y);
                    gr += g.re;
                    gi += g.im;
                }
                al = group16_sum(al);
                be = group16_sum(be);
                gr = group16_sum(gr);
                gi = group16_sum(gi);
                const double ga = sqrt(gr * gr + gi * gi);
                if (al <= small2 || be <= small2) continue;
                if (ga <= tol * sqrt(al) * sqrt(be)) continue;
                // phase e^{-i phi} on column q makes a_p^H a_q real positive
                const cplx ph = cmake(gr / ga, -gi / ga);
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = g16; i < m; i += 16) {
                    const cplx x = ap[i];
                    const cplx y = cmul(ph, aq[i]);
                    ap[i] = csub(cscale(x, c), cscale(y, s));
                    aq[i] = cadd(cscale(x, s), cscale(y, c));
                }
                if (g16 == 0 && fabs(t) > tmin) *flag = 1;
            }
            __syncthreads();
        }
        const int any = *flag;
        __syncthreads();
        if (!any) break;
    }
}

// Householder QR with column pivoting of the m x m column-major A in place,
// A P = Q R, leaving R^H (lower triangular) in A and the pivot order in perm
// (column j of A P is column perm[j] of A).  Q is never formed.  One group
// of 16 lanes per column (DPP sums inside the group): each group rebuilds
// the reflector of step j from column j (all groups compute the same bits),
// applies it to its trailing columns and recomputes their trailing norms
// exactly (cn, m doubles) for the next pivot search; two barriers per step.
__device__ void qrcp_to_rh(int m, cplx* A, int* perm, double* cn) {
    const int g16 = threadIdx.x & 15, group = threadIdx.x >> 4, ngroups = blockDim.x >> 4;
    for (int c = group; c < m; c += ngroups) {
        double sq = 0.0;
        for (int i = g16; i < m; i += 16) sq += cabs2(A[(long)c * m + i]);
        sq = group16_sum(sq);
        if (g16 == 0) cn[c] = sq;
    }
    for (int c = threadIdx.x; c < m; c += blockDim.x) perm[c] = c;
    __syncthreads();
    double beta_prev = 0.0;
    for (int j = 0; j < m; ++j) {
        // R(j-1, j-1): column j-1 is no longer read
        if (j > 0 && threadIdx.x == 0) A[(long)(j - 1) * m + (j - 1)] = cmake(beta_prev, 0.0);
        // pivot: the largest remaining trailing norm (ties: lowest index)
        double bv = -1.0;
        int bi = j;
        for (int c = j + g16; c < m; c += 16) {
            const double v = cn[c];
            if (v > bv) {
                bv = v;
                bi = c;
            }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, 16);
            const int oi = __shfl_xor(bi, o, 16);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        const int pj = bi;
        if (pj != j) {
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const cplx a = A[(long)j * m + i];
                A[(long)j * m + i] = A[(long)pj * m + i];
                A[(long)pj * m + i] = a;
            }
            if (threadIdx.x == 0) {
                const int t = perm[j];
                perm[j] = perm[pj];
                perm[pj] = t;
            }
        }
        __syncthreads();
        // reflector H = I - tau v v^H with v_j = 1, v_i = sc * A(i, j) (i > j)
        const cplx* col = A + (long)j * m;
        double s2 = 0.0;
        for (int i = j + 1 + g16; i < m; i += 16) s2 += cabs2(col[i]);
        s2 = group16_sum(s2);
        const cplx alpha = col[j];
        cplx tau = cmake(0, 0), sc = cmake(0, 0);
        double beta = alpha.re;
        if (!(s2 == 0.0 && alpha.im == 0.0)) {
            const double nrm = sqrt(cabs2(alpha) + s2);
            beta = alpha.re >= 0 ? -nrm : nrm;
            tau = cmake((beta - alpha.re) / beta, -alpha.im / beta);
            const cplx den = cmake(alpha.re - beta, alpha.im);
            const double dn = cabs2(den);
            sc = cmake(den.re / dn, -den.im / dn);
        }
        beta_prev = beta;
        const bool reflect = tau.re != 0.0 || tau.im != 0.0;
        const cplx ct = cconj(tau);
        for (int c = j + 1 + group; c < m; c += ngroups) {
            cplx* ac = A + (long)c * m;
            if (reflect) {
                double wr = 0.0, wi = 0.0;
                for (int i = j + g16; i < m; i += 16) {
                    const cplx v = (i == j) ? cmake(1, 0) : cmul(sc, col[i]);
                    const cplx t = cdotc(v, ac[i]);
                    wr += t.re;
                    wi += t.im;
                }
                wr = group16_sum(wr);
                wi = group16_sum(wi);
                const cplx f = cmul(ct, cmake(wr, wi));
                double sq = 0.0;
                for (int i = j + g16; i < m; i += 16) {
                    const cplx v = (i == j) ? cmake(1, 0) : cmul(sc, col[i]);
                    const cplx x = csub(ac[i], cmul(f, v));
                    ac[i] = x;
                    if (i > j) sq += cabs2(x);
                }
                sq = group16_sum(sq);
                if (g16 == 0) cn[c] = sq;
            } else if (g16 == 0) {
                cn[c] -= cabs2(ac[j]);  // only orders the pivots
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) A[(long)(m - 1) * m + (m - 1)] = cmake(beta_prev, 0.0);
    __syncthreads();
    // R (upper triangle) -> R^H (lower triangle), zeros above the diagonal
    for (long e = threadIdx.x; e < (long)m * m; e += blockDim.x) {
        const int c = (int)(e / m), r = (int)(e % m);
        if (r > c) {  // pair (c, r): R(c, r) sits at A[r][c]
            const cplx x = A[(long)r * m + c];
            A[(long)c * m + r] = cconj(x);
            A[(long)r * m + c] = cmake(0, 0);
        }
    }
    __syncthreads();
}

template <bool THETA_LDS>
__global__ __launch_bounds__(1024) void k_su_bond(SuDims dm, LayerDesc L, cplx* gam,
                                                  double* lam, double* eps, const cplx* gates,
                                                  char* scratch, size_t scratch_per_bond, JobMap jm) {
    // block row y: job y of jm (its tensors, weights, gates and scratch)
    gam = jptr(gam, jm, blockIdx.y);
    lam = jptr(lam, jm, blockIdx.y);
    eps = jptr(eps, jm, blockIdx.y);
    gates = jptr(gates, jm, blockIdx.y);
    scratch = jptr(scratch, jm, blockIdx.y);
    extern __shared__ char smem_raw[];
    __shared__ double red[16];
    __shared__ cplx bcast[2];
    __shared__ int flag;
    __shared__ int g_s;
    __shared__ double lam_inv_i[3][8], lam_inv_j[3][8], lam_i[3][8], lam_j[3][8];
    __shared__ double sig_sorted[512];  // also the pivoting norms of the QR
    __shared__ int col_of_rank[512];
    __shared__ int col_perm[512];

    const BondDesc bd = L.bond[blockIdx.x];
    const int D = dm.D, d = dm.d, Dc = dm.Dc, nb = dm.nb, r = dm.r, m = dm.m;
    SuScratch S;
    su_layout(dm, scratch + blockIdx.x * scratch_per_bond, &S);
    cplx* Ac = THETA_LDS ? (cplx*)smem_raw : S.Ac;
    const cplx* G = gates + (long)L.gate * d * d * d * d;
    const long site_sz = (long)d * D * D * D * D;
    cplx* gi = gam + bd.site_i * site_sz;
    cplx* gj = gam + bd.site_j * site_sz;

    // ---- outer lambdas and their pseudo-inverses (cutoff 1e-14 relative)
    if (threadIdx.x < 6) {
        const int side = threadIdx.x / 3, k = threadIdx.x % 3;
        const double* lv = lam + (long)(side ? bd.outer_j[k] : bd.outer_i[k]) * D;
        double mx = 0;
        for (int a = 0; a < D; ++a) mx = fmax(mx, lv[a]);
        for (int a = 0; a < D; ++a) {
            const double v = lv[a];
            (side ? lam_j : lam_i)[k][a] = v;
            (side ? lam_inv_j : lam_inv_i)[k][a] = (v > 1e-14 * mx) ? 1.0 / v : 0.0;
        }
    }
    __syncthreads();

    // ---- M_X = Gamma_X * outer lambdas, column-major (Dc x nb), col = s*D + b
    for (long e = threadIdx.x; e < (long)Dc * nb; e += blockDim.x) {
        const int col = (int)(e / Dc), row = (int)(e % Dc);
        const int s = col / D, b = col % D;
        const int o0 = row / (D * D), o1 = (row / D) % D, o2 = row % D;
        const double wi = lam_i[0][o0] * lam_i[1][o1] * lam_i[2][o2];
        const double wj = lam_j[0][o0] * lam_j[1][o1] * lam_j[2][o2];
        S.Mi[e] = cscale(gi[gam_offset(D, bd.leg_i, row, s, b)], wi);
        S.Mj[e] = cscale(gj[gam_offset(D, bd.leg_j, row, s, b)], wj);
    }
    __syncthreads();
    householder_qr(Dc, nb, r, S.Mi, S.taui, red, bcast);
    householder_qr(Dc, nb, r, S.Mj, S.tauj, red, bcast);

    // ---- Theta' (m x m, column-major), rows (k_i, s_i'), cols (s_j', k_j)
    const double* lb = lam + (long)bd.lam_b * D;
    for (long e = threadIdx.x; e < (long)m * m; e += blockDim.x) {
        const int col = (int)(e / m), row = (int)(e % m);
        const int ki = row / d, sip = row % d, sjp = col / r, kj = col % r;
        cplx acc = cmake(0, 0);
        for (int b = 0; b < D; ++b) {
            const double lv = lb[b];
            if (lv == 0.0) continue;
            for (int si = 0; si < d; ++si) {
                const int ci = si * D + b;
                if (ci < ki) continue;  // R_i is upper triangular
                const cplx ri = S.Mi[(long)ci * Dc + ki];
                for (int sj = 0; sj < d; ++sj) {
                    const int cj = sj * D + b;
                    if (cj < kj) continue;
                    const cplx rj = S.Mj[(long)cj * Dc + kj];
                    const cplx g = G[(sip * d + sjp) * d * d + si * d + sj];
                    acc = cadd(acc, cscale(cmul(g, cmul(ri, rj)), lv));
                }
            }
        }
        Ac[e] = acc;
        S.Th[e] = acc;
    }
    __syncthreads();
    // QR-preconditioned Jacobi: Theta' P = Q R, then one-sided Jacobi on the
    // columns of R^H (the rows of R, graded by the pivoting), which converge
    // in a few sweeps: R^H W = U~ S gives Theta' = (Q W) S (P U~)^H
    qrcp_to_rh(m, Ac, col_perm, sig_sorted);
    complex_jacobi(m, m, Ac, &flag, red);
    __syncthreads();

    // ---- singular values, ranks, truncation
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        double s = 0;
        for (int i = 0; i < m; ++i) s += cabs2(Ac[(long)c * m + i]);
        S.sig[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        const double sc = S.sig[c];
        int rank = 0;
        for (int l = 0; l < m; ++l) {
            const double sl = S.sig[l];
            rank += (sl > sc) || (sl == sc && l < c);
        }
        sig_sorted[rank] = sc;
        col_of_rank[rank] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0;
        for (int k = 0; k < m; ++k) tot += sig_sorted[k] * sig_sorted[k];
        if (!isfinite(tot)) {
            // non-finite input: poison the bond weights so the host notices
            for (int k = 0; k < D; ++k) lam[(long)bd.lam_b * D + k] = NAN;
            eps[bd.site_i] = NAN;
            eps[bd.site_j] = NAN;
            tot = 0.0;
        }
        int g = 0;
        if (sig_sorted[0] > 0) {
            int rk = 0;
            for (int k = 0; k < m; ++k) rk += sig_sorted[k] > 1e-12 * sig_sorted[0];
            g = rk < D ? rk : D;
            if (g < rk)
                while (g > 1 && sig_sorted[g - 1] - sig_sorted[g] <=
                                    1e-10 * sig_sorted[g - 1] + 1e-12 * sig_sorted[0])
                    --g;
        }
        double kept = 0;
        for (int k = 0; k < g; ++k) kept += sig_sorted[k] * sig_sorted[k];
        const double nk = sqrt(kept);
        if (tot > 0) {
            for (int k = 0; k < D; ++k) lam[(long)bd.lam_b * D + k] = (k < g) ? sig_sorted[k] / nk : 0.0;
            const double e = (tot - kept) / tot;
            eps[bd.site_i] += e;
            eps[bd.site_j] += e;
        }
        g_s = g;
    }
    __syncthreads();
    const int g = g_s;

    // ---- right vectors V_k = P (column / s_k), stored as B_k = V_k^H; left
    // vectors U_k = Theta' V_k / s_k  (k < g)
    for (long e = threadIdx.x; e < (long)m * g; e += blockDim.x) {
        const int k = (int)(e / m), i = (int)(e % m);
        S.B[(long)k * m + col_perm[i]] = cconj(cscale(Ac[(long)col_of_rank[k] * m + i], 1.0 / sig_sorted[k]));
    }
    __syncthreads();
    for (long e = threadIdx.x; e < (long)m * g; e += blockDim.x) {
        const int k = (int)(e / m), x = (int)(e % m);
        cplx acc = cmake(0, 0);
        for (int y = 0; y < m; ++y) acc = cadd(acc, cmul(S.Th[(long)y * m + x], cconj(S.B[(long)k * m + y])));
        S.U[(long)k * m + x] = cscale(acc, 1.0 / sig_sorted[k]);
    }
    __syncthreads();

    // ---- X_i = [U_g] (r rows used), X_j = [B_g], both Dc x nb, col = s*D + k
    for (long e = threadIdx.x; e < (long)Dc * nb; e += blockDim.x) {
        const int col = (int)(e / Dc), row = (int)(e % Dc);
        const int s = col / D, k = col % D;
        cplx xi = cmake(0, 0), xj = cmake(0, 0);
        if (row < r && k < g) {
            xi = S.U[(long)k * m + row * d + s];
            xj = S.B[(long)k * m + s * r + row];
        }
        S.Xi[e] = xi;
        S.Xj[e] = xj;
    }
    __syncthreads();
    householder_apply_q(Dc, r, nb, S.Mi, S.taui, S.Xi);
    householder_apply_q(Dc, r, nb, S.Mj, S.tauj, S.Xj);

    // ---- divide the outer lambdas back out, normalise to max |.| = 1, store
    for (int side = 0; side < 2; ++side) {
        cplx* X = side ? S.Xj : S.Xi;
        double mx = 0;
        for (long e = threadIdx.x; e < (long)Dc * nb; e += blockDim.x) {
            const int row = (int)(e % Dc);
            const int o0 = row / (D * D), o1 = (row / D) % D, o2 = row % D;
            const double w = side ? lam_inv_j[0][o0] * lam_inv_j[1][o1] * lam_inv_j[2][o2]
                                  : lam_inv_i[0][o0] * lam_inv_i[1][o1] * lam_inv_i[2][o2];
            const cplx v = cscale(X[e], w);
            X[e] = v;
            mx = fmax(mx, sqrt(cabs2(v)));
        }
        mx = block_max(mx, red);
        const double inv = mx > 0 ? 1.0 / mx : 0.0;
        cplx* gout = side ? gj : gi;
        const int leg = side ? bd.leg_j : bd.leg_i;
        for (long e = threadIdx.x; e < (long)Dc * nb; e += blockDim.x) {
            const int col = (int)(e / Dc), row = (int)(e % Dc);
            gout[gam_offset(D, leg, row, col / D, col % D)] = cscale(X[e], inv);
        }
        __syncthreads();
    }
}

void su_layer(hipStream_t s, int D, int d, const LayerDesc& L, cplx* gam, double* lam,
              double* eps, const cplx* gates, void* scratch, JobMap jm) {
    jm.per_job = 1;
    const dim3 grid(2, jm.delta ? jm.njobs : 1);
    const SuDims dm = su_dims(D, d);
    IPEPS_REQUIRE(dm.m <= 512 && D <= 8, IPEPS_EINVAL, "simple update: d*min(D^3,dD) > 512");
    const size_t per_bond = su_layout(dm, nullptr, nullptr);
    const size_t lds = (size_t)dm.m * dm.m * sizeof(cplx);
    static const size_t kMax = 160 * 1024 - 12 * 1024;
    if (lds <= kMax) {
        static bool attr = false;
        if (!attr) {
            HIP_CHECK(hipFuncSetAttribute((const void*)k_su_bond<true>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMax));
            attr = true;
        }
        hipLaunchKernelGGL(k_su_bond<true>, grid, dim3(1024), lds, s, dm, L, gam, lam, eps,
                           gates, (char*)scratch, per_bond, jm);
    } else {
        hipLaunchKernelGGL(k_su_bond<false>, grid, dim3(1024), 0, s, dm, L, gam, lam, eps,
                           gates, (char*)scratch, per_bond, jm);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace ipeps
