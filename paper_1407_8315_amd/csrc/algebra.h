// Small dense FP64 algebra for the per-bin decoder (one lane per bin).
//
// Everything works on de-rotated syndromes mt_l = e^{-i 2 pi k l / N} m_l, for
// which a bin holding values b_t at locations k + t M satisfies
//     mt_l = sum_t b_t w_d^{t l},   w_d = e^{i 2 pi / d}
// (Eq. (3) with z_j = e^{i 2 pi (k + t_j M) / N} = e^{i 2 pi k / N} w_d^{t_j}),
// so every bin is the same problem on the d-th roots of unity.
#pragma once

#include "common.h"

namespace sft {

// Singular values (descending) of the L x L Hankel matrix H_ij = mt_{i+j}
// (the matrix of Eq. (5) / Pruning Step 1), by one-sided Jacobi rotations on
// its columns: rotate column pairs until they are orthogonal; the column
// norms are then the singular values.  Full relative accuracy in FP64.
__host__ __device__ inline void hankel_singular_values(const zd* mt, int L, double* sv) {
    zd h[kMaxL][kMaxL];   // h[col][row]
#pragma unroll
    for (int j = 0; j < kMaxL; ++j)
#pragma unroll
        for (int i = 0; i < kMaxL; ++i) h[j][i] = (i < L && j < L) ? mt[i + j] : zd{0.0, 0.0};
    for (int sweep = 0; sweep < 12; ++sweep) {
        bool rotated = false;
#pragma unroll
        for (int p = 0; p < kMaxL - 1; ++p) {
#pragma unroll
            for (int q = p + 1; q < kMaxL; ++q) {
                if (q >= L) continue;
                double al = 0.0, be = 0.0;
                zd ga{0.0, 0.0};
#pragma unroll
                for (int i = 0; i < kMaxL; ++i) {
                    al += norm2(h[p][i]);
                    be += norm2(h[q][i]);
                    ga = ga + cmul_conj(h[p][i], h[q][i]);
                }
                // rotate unless |ga| <= 1e-16 sqrt(al be) (columns orthogonal to
                // working precision); squared test, one reciprocal for e and zeta
                const double g2 = norm2(ga);
                if (!(g2 > 1e-32 * (al * be)) || g2 == 0.0) continue;
                rotated = true;
                const double ag = sqrt(g2), rag = 1.0 / ag;
                const double zeta = (be - al) * (0.5 * rag);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                const zd e = zd{ga.x * rag, -ga.y * rag};   // e^{-i phi}, phi = arg(ga)
#pragma unroll
                for (int i = 0; i < kMaxL; ++i) {
                    zd hp = h[p][i], hq = e * h[q][i];
                    h[p][i] = c * hp - s * hq;
                    h[q][i] = s * hp + c * hq;
                }
            }
        }
        if (!rotated) break;
    }
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        double s2 = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxL; ++i) s2 += norm2(h[j][i]);
        sv[j] = (j < L) ? sqrt(s2) : 0.0;
    }
    // sort descending (L <= 4)
#pragma unroll
    for (int i = 0; i < kMaxL; ++i)
#pragma unroll
        for (int j = 0; j < kMaxL - 1; ++j)
            if (sv[j] < sv[j + 1]) {
                double tmp = sv[j];
                sv[j] = sv[j + 1];
                sv[j + 1] = tmp;
            }
}

// Singular values (descending) of the same Hankel matrix as the square roots
// of the eigenvalues of its Gram matrix G = H^H H (Hermitian, L x L), by
// cyclic two-sided Jacobi rotations on G.  About half the arithmetic of the
// one-sided sweeps, at the cost of absolute accuracy eps * sigma_1^2 in
// sigma^2 (a sigma of 1e-4 sigma_1 carries a relative error near 5e-9): used
// for the general-mode vote, which ranks singular values at noise level or
// above across bins, not for the rank test of exact mode.
__host__ __device__ inline void gram_singular_values(const zd* mt, int L, double* sv) {
    // upper triangle of G (g[i][j], j >= i; the diagonal is real), the lower
    // half being its conjugate
    zd g[kMaxL][kMaxL];
#pragma unroll
    for (int i = 0; i < kMaxL; ++i)
#pragma unroll
        for (int j = i; j < kMaxL; ++j) {
            zd acc{0.0, 0.0};
#pragma unroll
            for (int r = 0; r < kMaxL; ++r)
                if (r < L && j < L) acc = acc + (i == j ? zd{norm2(mt[r + i]), 0.0} : cmul_conj(mt[r + i], mt[r + j]));
            g[i][j] = acc;
        }
    // entry (r, c) of G from the stored triangle
    auto at = [&](int r, int c) -> zd { return r <= c ? g[r][c] : conj(g[c][r]); };
    for (int sweep = 0; sweep < 12; ++sweep) {
        bool rotated = false;
#pragma unroll
        for (int p = 0; p < kMaxL - 1; ++p) {
#pragma unroll
            for (int q = p + 1; q < kMaxL; ++q) {
                if (q >= L) continue;
                const double a = g[p][p].x, b = g[q][q].x;
                const zd ga = g[p][q];
                const double c2 = norm2(ga);
                if (!(c2 > 1e-32 * fabs(a * b)) || c2 == 0.0) continue;
                rotated = true;
                // with D = b - a, the rotation's tangent over |ga| is
                // tau = 2 sgn(D) / (|D| + sqrt(D^2 + 4 |ga|^2)) (the smaller
                // root), its cosine cs = (1 + tau^2 |ga|^2)^{-1/2};
                // U = [[cs, psi], [-conj(psi), cs]] on (p, q), psi = cs tau ga,
                // takes G to U^H G U with a zero at (p, q)
                const double dd = b - a;
#ifdef __HIP_DEVICE_COMPILE__
                // sqrt(q) = q q^{-1/2} and 1/h by the hardware reciprocal with
                // two Newton steps: tau to a few ulps, which only moves the
                // rotation angle; the rotation stays unitary to rounding since
                // cs is computed from the tau actually used
                const double qq = fma(dd, dd, 4.0 * c2);
                const double h = fabs(dd) + qq * rsqrt(qq);
                double y = __builtin_amdgcn_rcp(h);
                y = fma(fma(-h, y, 1.0), y, y);
                y = fma(fma(-h, y, 1.0), y, y);
                const double tau = (dd >= 0.0 ? 2.0 : -2.0) * y;
                const double tc = tau * c2;
                const double cs = rsqrt(1.0 + tau * tc);
#else
                const double tau = (dd >= 0.0 ? 2.0 : -2.0) / (fabs(dd) + sqrt(dd * dd + 4.0 * c2));
                const double tc = tau * c2;
                const double cs = 1.0 / sqrt(1.0 + tau * tc);
#endif
                const zd psi = (cs * tau) * ga;
#pragma unroll
                for (int r = 0; r < kMaxL; ++r) {
                    if (r == p || r == q || r >= L) continue;
                    const zd grp = at(r, p), grq = at(r, q);
                    const zd np = cs * grp - cmul_conj(psi, grq);   // cs G_rp - conj(psi) G_rq
                    const zd nq = psi * grp + cs * grq;
                    if (r < p) g[r][p] = np; else g[p][r] = conj(np);
                    if (r < q) g[r][q] = nq; else g[q][r] = conj(nq);
                }
                g[p][p] = zd{a - tc, 0.0};
                g[q][q] = zd{b + tc, 0.0};
                g[p][q] = zd{0.0, 0.0};
            }
        }
        if (!rotated) break;
    }
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) sv[j] = (j < L) ? sqrt(fmax(g[j][j].x, 0.0)) : 0.0;
#pragma unroll
    for (int i = 0; i < kMaxL; ++i)
#pragma unroll
        for (int j = 0; j < kMaxL - 1; ++j)
            if (sv[j] < sv[j + 1]) {
                double tmp = sv[j];
                sv[j] = sv[j + 1];
                sv[j + 1] = tmp;
            }
}

// a0 = #{sigma_i > tau_rank sigma_1}, at least 1.
__host__ __device__ inline int rank_order(const double* sv, int L, double tau_rank) {
    if (!(sv[0] > 0.0) || !__builtin_isfinite(sv[0])) return 1;
    int a = 0;
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) a += (i < L && sv[i] > tau_rank * sv[0]) ? 1 : 0;
    return a < 1 ? 1 : a;
}

// Exact shortcut of the rank test for bins of numerical rank one (most bins
// hold one frequency), which then skip the Jacobi sweeps.  R_ij = mt_i mt_j /
// mt_0 is a rank-one matrix, so sigma_2(H) <= ||H - R||_2 <= ||H - R||_F = dd
// (Eckart-Young) and sigma_1(H) >= sigma_1(R) - ||H - R||_2 >= rr - dd with
// rr = ||R||_F = ||R||_2.  dd (1 + tau) <= tau rr thus proves sigma_2 <=
// tau sigma_1, i.e. the rank test gives a0 = 1.  The margins cover the
// rounding of dd and rr and that of an SVD the decision is compared with.
// True only when a0 = 1 is certain (an all-zero bin also has a0 = 1); false
// means: run the SVD.
__host__ __device__ __attribute__((always_inline)) inline bool rank_one_certified(const zd* mt, int L, double tau_rank) {
    if (L == 1) return true;
    const double n0 = norm2(mt[0]);
    double e = 0.0;
#pragma unroll
    for (int l = 0; l < 2 * kMaxL - 1; ++l)
        if (l <= 2 * L - 2) e += norm2(mt[l]);
    if (e == 0.0) return true;
    if (!(n0 > 0.0) || !__builtin_isfinite(e)) return false;
    const zd inv0 = frcp(n0) * conj(mt[0]);
    zd u[kMaxL];
    double colsq = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) {
        u[i] = mt[i] * inv0;
        if (i < L) colsq += norm2(mt[i]);
    }
    double dd2 = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxL; ++i)
#pragma unroll
        for (int j = 0; j < kMaxL; ++j)
            if (i < L && j < L) dd2 += norm2(mt[i + j] - mt[i] * u[j]);
    const double rr = colsq / sqrt(n0), dd = sqrt(dd2);
    const double eps = 2.220446049250313e-16;
    return __builtin_isfinite(rr) && dd * (1.0 + tau_rank) * (1.0 + 1e-9) + 64.0 * eps * rr <= tau_rank * rr;
}

// Step (i): solve sum_j c_j mt_{i+j} = -mt_{a+i}, i < a (Eq. (5)), by Gaussian
// elimination with partial pivoting.  False when a pivot is zero or the
// solution is not finite.
__host__ __device__ __attribute__((always_inline)) inline bool locator(const zd* mt, int a, zd* c) {
    // Register arrays are only indexed by unrolled constants (a runtime index
    // would send them to scratch memory): the right-hand side and the pivot
    // row swap are written as predicated selections.
    zd A[kMaxL][kMaxL + 1];
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) {
#pragma unroll
        for (int j = 0; j < kMaxL; ++j) A[i][j] = (i < a && j < a) ? mt[i + j] : zd{0.0, 0.0};
        zd rhs{0.0, 0.0};
#pragma unroll
        for (int l = 0; l < 2 * kMaxL; ++l)
            if (i < a && l == a + i) rhs = -mt[l];
        A[i][kMaxL] = rhs;
    }
#pragma unroll
    for (int col = 0; col < kMaxL; ++col) {
        if (col >= a) break;
        int piv = col;
        double best = norm2(A[col][col]);
#pragma unroll
        for (int r = col + 1; r < kMaxL; ++r)
            if (r < a && norm2(A[r][col]) > best) {
                best = norm2(A[r][col]);
                piv = r;
            }
        if (!(best > 0.0)) return false;
#pragma unroll
        for (int r = col + 1; r < kMaxL; ++r) {
            if (r == piv) {
#pragma unroll
                for (int j = 0; j <= kMaxL; ++j) {
                    zd tmp = A[col][j];
                    A[col][j] = A[r][j];
                    A[r][j] = tmp;
                }
            }
        }
#pragma unroll
        for (int r = col + 1; r < kMaxL; ++r) {
            if (r >= a) break;
            zd f = cdiv(A[r][col], A[col][col]);
#pragma unroll
            for (int j = col; j <= kMaxL; ++j) A[r][j] = A[r][j] - f * A[col][j];
        }
    }
#pragma unroll
    for (int i = kMaxL - 1; i >= 0; --i) {
        if (i >= a) continue;
        zd s = A[i][kMaxL];
#pragma unroll
        for (int j = i + 1; j < kMaxL; ++j)
            if (j < a) s = s - A[i][j] * c[j];
        c[i] = cdiv(s, A[i][i]);
        if (!cfinite(c[i])) return false;
    }
    return true;
}

// P(z) = z^a + sum_j c_j z^j and P'(z) by Horner.
__host__ __device__ __attribute__((always_inline)) inline void poly_eval(const zd* c, int a, zd z, zd& p, zd& dp) {
    p = zd{1.0, 0.0};
    dp = zd{0.0, 0.0};
#pragma unroll
    for (int j = kMaxL - 1; j >= 0; --j) {
        if (j < a) {
            dp = dp * z + p;
            p = p * z + c[j];
        }
    }
}

// Step (ii): the a roots of P.  a = 1: -c_0.  a = 2: the quadratic formula in
// its cancellation-free form.  a = 3, 4: Aberth-Ehrlich simultaneous
// iterations from points spread on the unit circle (the roots of a decodable
// bin lie on it).  False if an iteration does not converge.
__host__ __device__ __attribute__((always_inline)) inline bool poly_roots(const zd* c, int a, zd* z) {
    if (a == 1) {
        z[0] = -c[0];
        return cfinite(z[0]);
    }
    if (a == 2) {
        zd disc = c[1] * c[1] - 4.0 * c[0];
        zd s = csqrt(disc);
        if (c[1].x * s.x + c[1].y * s.y < 0.0) s = -s;   // Re(conj(c1) s) >= 0
        zd q = -0.5 * (c[1] + s);
        if (norm2(q) == 0.0) {
            z[0] = z[1] = zd{0.0, 0.0};
            return true;
        }
        z[0] = q;
        z[1] = cdiv(c[0], q);
        return cfinite(z[0]) && cfinite(z[1]);
    }
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        const double ang = M_PI * (2.0 * j / a + 0.123);
        z[j] = zd{cos(ang), sin(ang)};
    }
    // Stop when the largest correction is below 1e-10 (relative); near a
    // cluster of roots rounding keeps the corrections around eps / spacing^(a-1),
    // so after the iteration cap a final correction below 1e-7 is accepted
    // (the grid check that follows needs far less than that: it compares the
    // root's angle with the grid spacing, at least 2 pi / 2^22).
    double step = 0.0;
    for (int it = 0; it < 40; ++it) {
        double scale = 0.0;
        step = 0.0;
        bool bad = false;
#pragma unroll
        for (int j = 0; j < kMaxL; ++j) {
            if (j >= a) continue;
            zd p, dp;
            poly_eval(c, a, z[j], p, dp);
            if (norm2(p) == 0.0) continue;
            // Aberth correction (p/p') / (1 - (p/p') sum_k 1/(z_j - z_k)),
            // written as p / (p' - p sum_k 1/(z_j - z_k)): one division per
            // term (the magnitudes here stay far from overflow).
            zd sum{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                if (k < a && k != j) {
                    const zd dz = z[j] - z[k];
                    sum = sum + frcp(norm2(dz)) * conj(dz);
                }
            const zd den = dp - p * sum;
            zd w = frcp(norm2(den)) * (p * conj(den));
            bad |= !cfinite(w);
            z[j] = z[j] - w;
            step = fmax(step, norm2(w));
            scale = fmax(scale, norm2(z[j]));
        }
        if (bad) return false;
        if (step <= 1e-20 * fmax(scale, 1.0)) return true;
    }
    return step <= 1e-14;
}

// Alg. 1 grid check on de-rotated roots: z_j must lie within delta_mag of the
// unit circle and within delta_grid grid spacings of w_d^{t_j}; the t_j must be
// distinct.  Writes t_j in [0, d).
__host__ __device__ __attribute__((always_inline)) inline bool roots_to_grid(const zd* z, int a, int64_t d, double delta_grid, double delta_mag,
                                     int64_t* t) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        if (j >= a) continue;
        double mag = cabs(z[j]);
        ok &= fabs(mag - 1.0) <= delta_mag;
        double u = atan2(z[j].y, z[j].x) * ((double)d / (2.0 * M_PI));
        double r = floor(u + 0.5);
        ok &= fabs(u - r) <= delta_grid;
        const int64_t tt = (int64_t)r & (d - 1);   // r mod d (d is a power of two)
#pragma unroll
        for (int k = 0; k < kMaxL; ++k)
            if (k < j) ok &= t[k] != tt;
        t[j] = tt;
    }
    return ok;
}

// Solve the Hermitian positive definite system G x = b (n <= NMAX) in place by
// Cholesky on the packed lower triangle.  False when not positive definite.
// Each pivot takes one reciprocal square root r_j = d_j^{-1/2}: L_jj = d_j r_j,
// and the column scaling and both substitutions multiply by r_j.
template <int NMAX>
__host__ __device__ __attribute__((always_inline)) inline bool chol_solve(zd (&g)[NMAX * (NMAX + 1) / 2], zd* b, int n) {
    // g holds rows i >= j at index i*(i+1)/2 + j
    double rinv[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        rinv[j] = 1.0;
        if (j >= n) break;
        double dj = g[j * (j + 1) / 2 + j].x;
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k < j) dj -= norm2(g[j * (j + 1) / 2 + k]);
        if (!(dj > 0.0)) return false;
#ifdef __HIP_DEVICE_COMPILE__
        const double rj = rsqrt(dj);
#else
        const double rj = 1.0 / sqrt(dj);
#endif
        rinv[j] = rj;
        g[j * (j + 1) / 2 + j] = zd{dj * rj, 0.0};
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            if (i <= j || i >= n) continue;
            zd s = g[i * (i + 1) / 2 + j];
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < j) s = s - g[i * (i + 1) / 2 + k] * conj(g[j * (j + 1) / 2 + k]);
            g[i * (i + 1) / 2 + j] = rj * s;
        }
    }
    // forward: L y = b
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        if (i >= n) break;
        zd s = b[i];
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k < i) s = s - g[i * (i + 1) / 2 + k] * b[k];
        b[i] = rinv[i] * s;
    }
    // backward: L^H x = y
#pragma unroll
    for (int i = NMAX - 1; i >= 0; --i) {
        if (i >= n) continue;
        zd s = b[i];
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k > i && k < n) s = s - conj(g[k * (k + 1) / 2 + i]) * b[k];
        b[i] = rinv[i] * s;
    }
    return true;
}

// w_d^q from the plan's FP64 table (q reduced mod d by the caller).
__host__ __device__ __attribute__((always_inline)) inline zd omega(const double2* tab, int stride, int64_t q) {
    double2 v = tab[q * stride];
    return zd{v.x, v.y};
}

// Step (iii): p = argmin ||V p - mt|| over the first `rows` syndromes with
// V_lj = w_j^l, w_j = w_d^{t_j}, by the normal equations; returns the residual
// energy.  Columns are generated as running powers (rows <= 8 products each),
// so V is never stored.  mt has 2 kMaxL entries (zero beyond `rows`).
__host__ __device__ __attribute__((always_inline)) inline bool vandermonde_ls(const zd* mt, int rows, const int64_t* t, int a, int64_t d,
                                      const double2* tab, int stride, zd* p, double& r2) {
    (void)d;
    zd w[kMaxL], pw[kMaxL];
    zd g[kMaxL * (kMaxL + 1) / 2];
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        w[j] = (j < a) ? omega(tab, stride, t[j]) : zd{0.0, 0.0};
        pw[j] = zd{1.0, 0.0};
        p[j] = zd{0.0, 0.0};
    }
    // right-hand side V^H mt
#pragma unroll
    for (int l = 0; l < 2 * kMaxL; ++l) {
        if (l >= rows) break;
#pragma unroll
        for (int j = 0; j < kMaxL; ++j) {
            if (j >= a) continue;
            p[j] = p[j] + cmul_conj(pw[j], mt[l]);
            pw[j] = pw[j] * w[j];
        }
    }
    // Gram matrix G_ij = sum_l (conj(w_i) w_j)^l
#pragma unroll
    for (int i = 0; i < kMaxL; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            if (i >= a) continue;
            zd q = cmul_conj(w[i], w[j]), acc{0.0, 0.0}, pq{1.0, 0.0};
#pragma unroll
            for (int l = 0; l < 2 * kMaxL; ++l) {
                if (l >= rows) break;
                acc = acc + pq;
                pq = pq * q;
            }
            g[i * (i + 1) / 2 + j] = acc;
        }
    if (!chol_solve<kMaxL>(g, p, a)) return false;
    r2 = 0.0;
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) pw[j] = zd{1.0, 0.0};
#pragma unroll
    for (int l = 0; l < 2 * kMaxL; ++l) {
        if (l >= rows) break;
        zd e = mt[l];
#pragma unroll
        for (int j = 0; j < kMaxL; ++j) {
            if (j >= a) continue;
            e = e - pw[j] * p[j];
            pw[j] = pw[j] * w[j];
        }
        r2 += norm2(e);
    }
    bool ok = __builtin_isfinite(r2);
#pragma unroll
    for (int j = 0; j < kMaxL; ++j)
        if (j < a) ok &= cfinite(p[j]);
    return ok;
}

}  // namespace sft
