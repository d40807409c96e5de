/*
 * Plain-C inner loops of the CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Only the oracle package loads this file's shared object; the product path
 * never links it.  Everything here is deliberately simple: unsigned __int128
 * products and '%' reductions, no blocking, no fusion.
 *
 *  orc_rinv     right inverse of a matrix over Z/q, q = p^M, found by
 *               Gauss-Jordan elimination with unit pivots (a pivot is a unit
 *               iff it is nonzero mod p).  Used for the decomposition map of
 *               Proposition 3.3 and for the Griffiths-Dwork solves of
 *               Section 3.3, step (2).
 *  orc_reduce   controlled reduction of start terms one pole order at a time
 *               (Proposition 3.3 with the explicit R_{u,v}(g) of Section 3.1,
 *               written as polynomial arithmetic), with v chosen by the
 *               greedy Algorithm 3 at every step.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * b) % q);
}

static uint64_t invmod(uint64_t a, uint64_t q) {
    /* extended Euclid on signed 128-bit values; a must be a unit mod q */
    __int128 t = 0, nt = 1, r = (__int128)q, nr = (__int128)(a % q);
    while (nr != 0) {
        __int128 qq = r / nr, tmp;
        tmp = t - qq * nt; t = nt; nt = tmp;
        tmp = r - qq * nr; r = nr; nr = tmp;
    }
    if (r != 1) return 0;
    if (t < 0) t += (__int128)q;
    return (uint64_t)t;
}

/*
 * A: rows x cols (row-major) over Z/q.  out: cols x rows with A*out = I.
 * Columns are scanned left to right; a column becomes a pivot column when one
 * of the not-yet-used rows holds a unit in it.  Returns the rank found; the
 * caller treats rank < rows as "not surjective mod p".
 */
int orc_rinv(int rows, int cols, const uint64_t *A, uint64_t q, uint64_t p,
             uint64_t *out) {
    int w = cols + rows;
    uint64_t *W = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)rows * w);
    int *piv = (int *)malloc(sizeof(int) * (rows > 0 ? rows : 1));
    for (int r = 0; r < rows; r++) {
        for (int c = 0; c < cols; c++) W[(size_t)r * w + c] = A[(size_t)r * cols + c] % q;
        for (int c = 0; c < rows; c++) W[(size_t)r * w + cols + c] = (r == c) ? 1 : 0;
    }
    int rank = 0;
    for (int c = 0; c < cols && rank < rows; c++) {
        int sel = -1;
        for (int r = rank; r < rows; r++)
            if (W[(size_t)r * w + c] % p != 0) { sel = r; break; }
        if (sel < 0) continue;
        if (sel != rank)
            for (int k = 0; k < w; k++) {
                uint64_t t = W[(size_t)sel * w + k];
                W[(size_t)sel * w + k] = W[(size_t)rank * w + k];
                W[(size_t)rank * w + k] = t;
            }
        uint64_t inv = invmod(W[(size_t)rank * w + c], q);
        for (int k = 0; k < w; k++) W[(size_t)rank * w + k] = mulmod(W[(size_t)rank * w + k], inv, q);
        for (int r = 0; r < rows; r++) {
            if (r == rank) continue;
            uint64_t f = W[(size_t)r * w + c];
            if (f == 0) continue;
            uint64_t nf = q - f;
            for (int k = 0; k < w; k++) {
                uint64_t x = W[(size_t)rank * w + k];
                if (x) W[(size_t)r * w + k] = (uint64_t)((W[(size_t)r * w + k] + (u128)nf * x) % q);
            }
        }
        piv[rank++] = c;
    }
    memset(out, 0, sizeof(uint64_t) * (size_t)cols * rows);
    if (rank == rows)
        for (int k = 0; k < rows; k++)
            for (int j = 0; j < rows; j++)
                out[(size_t)piv[k] * rows + j] = W[(size_t)k * w + cols + j];
    free(W);
    free(piv);
    return rank;
}

/* dense exponent -> index lookup over the first nv-1 exponents */
typedef struct {
    int nv, deg;
    int *tab;
} lookup_t;

static int lk_key(const lookup_t *L, const int *e) {
    int key = 0;
    for (int i = 0; i < L->nv - 1; i++) {
        if (e[i] < 0 || e[i] > L->deg) return -1;
        key = key * (L->deg + 1) + e[i];
    }
    return key;
}

static void lk_build(lookup_t *L, int nv, int deg, int count, const int *exps) {
    int size = 1;
    for (int i = 0; i < nv - 1; i++) size *= (deg + 1);
    L->nv = nv;
    L->deg = deg;
    L->tab = (int *)malloc(sizeof(int) * size);
    for (int i = 0; i < size; i++) L->tab[i] = -1;
    for (int k = 0; k < count; k++) L->tab[lk_key(L, exps + (size_t)k * nv)] = k;
}

static int lk_find(const lookup_t *L, const int *e) {
    int s = 0;
    for (int i = 0; i < L->nv; i++) {
        if (e[i] < 0) return -1;
        s += e[i];
    }
    if (s != L->deg) return -1;
    int key = lk_key(L, e);
    return key < 0 ? -1 : L->tab[key];
}

/* Algorithm 3 (greedy choice of v) with the loop ended as soon as |v| = d.
 * Returns 0 if the result is a valid direction for the current exponent U
 * (U - v >= 0 and, for i in S, U_i != 0 implies v_i != 0), -1 otherwise. */
static int greedy_v(int nv, int d, uint32_t Smask, const int *U, int *v) {
    int left = d;
    for (int i = 0; i < nv; i++) v[i] = 0;
    for (int s = 0; s < nv && left > 0; s++)
        if ((Smask >> s) & 1u)
            if (U[s] != 0) { v[s] = 1; left--; }
    while (left > 0) {
        int progressed = 0;
        for (int m = 0; m < nv && left > 0; m++)
            if (v[m] < U[m]) { v[m]++; left--; progressed = 1; }
        if (!progressed) return -1;
    }
    for (int i = 0; i < nv; i++) {
        if (U[i] - v[i] < 0) return -1;
        if (((Smask >> i) & 1u) && U[i] != 0 && v[i] == 0) return -1;
    }
    return 0;
}

/*
 * Reduce start blocks to pole order n and accumulate their pole-n numerators.
 *
 *   nv = n+1, d, Smask (bit i set <=> i in S), q = p^M
 *   g-space   Homog_{dn-n}            : s monomials  gexp[s*nv]
 *   tgt-space Homog_{D}, D=dn+d-n-|S| : T monomials  texp[T*nv]
 *   src       block i: Homog_{D-d+1} (i in S) or Homog_{D-d} (i not in S),
 *             nsrc monomials sexp[nsrc*nv], block id sblk[nsrc]
 *   psi       nsrc x T right inverse of the J_S map (row-major)
 *   fin-space Homog_{dn-n-1}          : F monomials  fexp[F*nv]
 *   nblk start blocks: exponent E'[nblk*nv] (numerator x^{E'}/x^S), pole P[nblk],
 *             coefficient rows coef[nblk*b]
 *   H         F x b output (row-major), accumulated mod q
 *   Jchk      optional T x nsrc matrix of J_S; when non-NULL every step checks
 *             J_S * (g_i) == x^v g / x^S exactly.
 * Returns 0, or a negative code on an invariant violation.
 */
int orc_reduce(int nv, int d, uint32_t Smask, uint64_t q,
               int s, const int *gexp, int T, const int *texp,
               int nsrc, const int *sexp, const int *sblk,
               const uint64_t *psi, int F, const int *fexp,
               int nblk, const int *Eexp, const int *P, int b,
               const uint64_t *coef, uint64_t *H, const uint64_t *Jchk) {
    int n = nv - 1, nS = 0;
    for (int i = 0; i < nv; i++) nS += (Smask >> i) & 1u;
    int D = d * n + d - n - nS;
    lookup_t Lg, Lt, Lf;
    lk_build(&Lg, nv, d * n - n, s, gexp);
    lk_build(&Lt, nv, D, T, texp);
    lk_build(&Lf, nv, d * n - n - 1, F, fexp);
    uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * s);
    uint64_t *g2 = (uint64_t *)malloc(sizeof(uint64_t) * s);
    uint64_t *h = (uint64_t *)malloc(sizeof(uint64_t) * T);
    uint64_t *G = (uint64_t *)malloc(sizeof(uint64_t) * nsrc);
    int *nz = (int *)malloc(sizeof(int) * T);
    int U[16], v[16], u[16], e[16];
    int rc = 0;
    for (int blk = 0; blk < nblk && rc == 0; blk++) {
        /* Algorithm 1: Tweak(E', dn-n) removes dn-n units from the front */
        const int *E = Eexp + (size_t)blk * nv;
        int left = d * n - n;
        int gam[16];
        for (int i = 0; i < nv; i++) {
            int take = E[i] < left ? E[i] : left;
            gam[i] = take;
            U[i] = E[i] - take;
            left -= take;
        }
        if (left != 0) { rc = -1; break; }
        memset(g, 0, sizeof(uint64_t) * s);
        int gi = lk_find(&Lg, gam);
        if (gi < 0) { rc = -2; break; }
        g[gi] = 1;
        for (int pole = P[blk]; pole > n; pole--) {
            if (greedy_v(nv, d, Smask, U, v) != 0) { rc = -3; break; }
            for (int i = 0; i < nv; i++) u[i] = U[i] - v[i];
            /* x^v g / x^S in Homog_D */
            memset(h, 0, sizeof(uint64_t) * T);
            int nnz = 0;
            for (int k = 0; k < s; k++) {
                if (!g[k]) continue;
                for (int i = 0; i < nv; i++)
                    e[i] = v[i] + gexp[(size_t)k * nv + i] - (int)((Smask >> i) & 1u);
                int t = lk_find(&Lt, e);
                if (t < 0) { rc = -4; break; }
                h[t] = (h[t] + g[k]) % q;
            }
            if (rc) break;
            for (int t = 0; t < T; t++)
                if (h[t]) nz[nnz++] = t;
            /* (g_i) = psi * h */
            for (int r = 0; r < nsrc; r++) {
                u128 acc = 0;
                const uint64_t *row = psi + (size_t)r * T;
                for (int k = 0; k < nnz; k++) {
                    acc += (u128)row[nz[k]] * h[nz[k]];
                    if (acc >> 125) acc %= q;
                }
                G[r] = (uint64_t)(acc % q);
            }
            if (Jchk) {
                for (int t = 0; t < T; t++) {
                    u128 acc = 0;
                    for (int r = 0; r < nsrc; r++) {
                        acc += (u128)Jchk[(size_t)t * nsrc + r] * G[r];
                        if (acc >> 125) acc %= q;
                    }
                    if ((uint64_t)(acc % q) != h[t]) { rc = -5; break; }
                }
                if (rc) break;
            }
            /* R_{u,v}(g) = x^S sum_{i in S} (u_i g_i + x_i d_i g_i)/x_i
             *            + x^S sum_{i not in S} ((u_i+1) g_i + x_i d_i g_i)       */
            memset(g2, 0, sizeof(uint64_t) * s);
            for (int r = 0; r < nsrc && rc == 0; r++) {
                if (!G[r]) continue;
                int i = sblk[r];
                const int *mu = sexp + (size_t)r * nv;
                int inS = (Smask >> i) & 1u;
                for (int j = 0; j < nv; j++) e[j] = mu[j] + (int)((Smask >> j) & 1u);
                if (inS) e[i] -= 1;
                int out = lk_find(&Lg, e);
                if (out < 0) { rc = -6; break; }
                /* term u_i g_i (divided by x_i when i in S, times (u_i+1) otherwise) */
                uint64_t w1 = (uint64_t)(u[i] + (inS ? 0 : 1));
                g2[out] = (uint64_t)((g2[out] + (u128)w1 * G[r]) % q);
                /* term x_i d_i g_i: the derivative brings down mu_i */
                g2[out] = (uint64_t)((g2[out] + (u128)(uint64_t)mu[i] * G[r]) % q);
            }
            if (rc) break;
            memcpy(g, g2, sizeof(uint64_t) * s);
            memcpy(U, u, sizeof(int) * nv);
        }
        if (rc) break;
        /* pole n: numerator x^U g / x^S in Homog_{dn-n-1} */
        for (int k = 0; k < s; k++) {
            if (!g[k]) continue;
            for (int i = 0; i < nv; i++)
                e[i] = U[i] + gexp[(size_t)k * nv + i] - (int)((Smask >> i) & 1u);
            int fi = lk_find(&Lf, e);
            if (fi < 0) { rc = -7; break; }
            for (int c = 0; c < b; c++) {
                uint64_t cc = coef[(size_t)blk * b + c];
                if (!cc) continue;
                H[(size_t)fi * b + c] = (uint64_t)((H[(size_t)fi * b + c] + (u128)cc * g[k]) % q);
            }
        }
    }
    free(Lg.tab); free(Lt.tab); free(Lf.tab);
    free(g); free(g2); free(h); free(G); free(nz);
    return rc;
}
