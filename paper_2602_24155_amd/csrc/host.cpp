// Host setup / finishing for controlled reduction (see host.hpp).
#include "host.hpp"
#include "device_layout.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>

namespace crf {

// ------------------------------------------------------------------ ModQ
void ModQ::init(u64 modulus) {
    q = modulus;
    sbits = 0;
    while (sbits < 64 && (modulus >> sbits) != 0) sbits++;
    mu = (u64)(((u128)1 << (2 * sbits + 8)) / q);
}

u64 ModQ::inv(u64 a) const {
    i128 t = 0, nt = 1, r = (i128)q, nr = (i128)(a % q);
    while (nr != 0) {
        i128 k = r / nr, tmp = t - k * nt;
        t = nt;
        nt = tmp;
        tmp = r - k * nr;
        r = nr;
        nr = tmp;
    }
    if (t < 0) t += (i128)q;
    return (u64)t;
}

// ------------------------------------------------------------------ monomials
long long binom(int n, int k) {
    if (k < 0 || n < 0 || k > n) return 0;
    long long r = 1;
    for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
    return r;
}

long long count_monomials(int nv, int deg) { return deg < 0 ? 0 : binom(deg + nv - 1, nv - 1); }

namespace {
// C(n, k) for 0 <= n < 96, 0 <= k <= 8 (monomial ranks of degree < 90 in <= 8 variables)
struct BinomTable {
    long long t[96][9];
    BinomTable() {
        for (int n = 0; n < 96; n++)
            for (int k = 0; k < 9; k++) t[n][k] = binom(n, k);
    }
};
const BinomTable &btab() {
    static const BinomTable T;
    return T;
}
}  // namespace

void MonoSpace::init(int nvars, int degree) {
    nv = nvars;
    deg = degree;
    count = (int)count_monomials(nv, deg);
    exps.assign((size_t)count * nv, 0);
    if (count == 0) return;
    // odometer over lex-descending exponent vectors
    std::vector<int> e(nv, 0);
    e[0] = deg;
    for (int k = 0; k < count; k++) {
        for (int i = 0; i < nv; i++) exps[(size_t)k * nv + i] = (int8_t)e[i];
        // next: find the rightmost position j < nv-1 with e[j] > 0, move one unit right
        int j = nv - 2;
        while (j >= 0 && e[j] == 0) j--;
        if (j < 0) break;
        e[j]--;
        int tail = 0;
        for (int i = j + 1; i < nv; i++) tail += e[i];
        for (int i = j + 1; i < nv; i++) e[i] = 0;
        e[j + 1] = tail + 1;
    }
}

int MonoSpace::rank(const int *e) const {
    int sum = 0;
    for (int i = 0; i < nv; i++) {
        if (e[i] < 0) return -1;
        sum += e[i];
    }
    if (sum != deg) return -1;
    // monomials before e: for each position i, those with the same prefix and a
    // larger exponent at i; sum_{t > e_i} count(nv-i-1, rem-t) = C(rem - e_i - 1 + k, k)
    // with k = nv - i - 1 (hockey-stick identity)
    const BinomTable &B = btab();
    long long idx = 0;
    int rem = deg;
    for (int i = 0; i < nv - 1; i++) {
        const int k = nv - i - 1, top = rem - e[i] - 1 + k;
        if (rem - e[i] > 0) idx += (top < 96 && k < 9) ? B.t[top][k] : binom(top, k);
        rem -= e[i];
    }
    return (int)idx;
}

// ------------------------------------------------------------------ family tables
bool Family::init(int nvars, int degree, uint32_t s_mask, std::string &err) {
    nv = nvars;
    n = nv - 1;
    d = degree;
    if (nv < 3 || nv > kMaxVars || d < 2) {
        err = "unsupported nvars/degree";
        return false;
    }
    smask = s_mask ? s_mask : ((1u << nv) - 1);
    if (smask >> nv) {
        err = "s_mask has bits beyond nvars";
        return false;
    }
    nS = __builtin_popcount(smask);
    if (d < nS) {
        err = "controlled reduction needs degree >= |S|";
        return false;
    }
    D = d * n + d - n - nS;
    coeff.init(nv, d);
    g.init(nv, d * n - n);
    tgt.init(nv, D);
    fin.init(nv, d * n - n - 1);
    dirs.init(nv, d);
    finU.init(nv, nS - 1);
    if (tgt.count > 32767 || g.count > 32767) {
        err = "index tables exceed 16-bit range";
        return false;
    }
    srcblk.resize(nv);
    srcoff.assign(nv + 1, 0);
    for (int i = 0; i < nv; i++) {
        bool inS = (smask >> i) & 1u;
        srcblk[i].init(nv, inS ? D - d + 1 : D - d);
        srcoff[i + 1] = srcoff[i] + srcblk[i].count;
    }
    nsrc = srcoff[nv];
    if (nsrc > 32767) {
        err = "index tables exceed 16-bit range";
        return false;
    }
    const int s = g.count;
    int e[kMaxVars];
    colmap.assign((size_t)dirs.count * s, -1);
    for (int v = 0; v < dirs.count; v++)
        for (int k = 0; k < s; k++) {
            for (int i = 0; i < nv; i++) e[i] = dirs.at(v)[i] + g.at(k)[i] - (int)((smask >> i) & 1u);
            colmap[(size_t)v * s + k] = (int16_t)tgt.rank(e);
        }
    gsrc.assign((size_t)s * nv, -1);
    gw.assign((size_t)s * nv, 0);
    for (int r = 0; r < s; r++)
        for (int i = 0; i < nv; i++) {
            bool inS = (smask >> i) & 1u;
            for (int j = 0; j < nv; j++) e[j] = g.at(r)[j] - (int)((smask >> j) & 1u) + ((inS && j == i) ? 1 : 0);
            int idx = srcblk[i].rank(e);
            gsrc[(size_t)r * nv + i] = (int16_t)(idx < 0 ? -1 : srcoff[i] + idx);
            gw[(size_t)r * nv + i] = (int16_t)(g.at(r)[i] + (inS ? 0 : 1));
        }
    finmap.assign((size_t)finU.count * s, -1);
    for (int U = 0; U < finU.count; U++)
        for (int k = 0; k < s; k++) {
            for (int i = 0; i < nv; i++) e[i] = finU.at(U)[i] + g.at(k)[i] - (int)((smask >> i) & 1u);
            finmap[(size_t)U * s + k] = (int16_t)fin.rank(e);
        }
    jtab.assign((size_t)tgt.count * nsrc, -1);
    for (int t = 0; t < tgt.count; t++)
        for (int i = 0; i < nv; i++) {
            const bool inS = (smask >> i) & 1u;
            for (int a = 0; a < srcblk[i].count; a++) {
                bool ok = true;
                for (int j = 0; j < nv; j++) {
                    e[j] = tgt.at(t)[j] - srcblk[i].at(a)[j];
                    ok = ok && e[j] >= 0;
                }
                if (!ok) continue;
                const int w = inS ? e[i] + 1 : e[i];
                if (inS) e[i] += 1;
                const int idx = coeff.rank(e);
                if (w > 0 && idx >= 0) jtab[(size_t)t * nsrc + srcoff[i] + a] = (idx << 8) | w;
            }
        }
    return true;
}

// ------------------------------------------------------------------ small helpers
static bool is_prime(int p) {
    if (p < 2) return false;
    for (int k = 2; k * k <= p; k++)
        if (p % k == 0) return false;
    return true;
}

static int vp_fact(long long x, int p) {
    int v = 0;
    for (long long t = p; t <= x; t *= p) v += (int)(x / t);
    return v;
}

// dense polynomial over one MonoSpace, coefficients mod q
struct DPoly {
    const MonoSpace *sp;
    std::vector<u64> c;
};

// exact unsigned big integer (base 2^32) for precision comparisons
struct Big {
    std::vector<uint32_t> w{1};
    void mul(uint64_t k) {
        u128 carry = 0;
        for (auto &x : w) {
            u128 t = (u128)x * k + carry;
            x = (uint32_t)t;
            carry = t >> 32;
        }
        while (carry) {
            w.push_back((uint32_t)carry);
            carry >>= 32;
        }
    }
    static int cmp(const Big &a, const Big &b) {
        size_t na = a.w.size(), nb = b.w.size();
        while (na > 1 && a.w[na - 1] == 0) na--;
        while (nb > 1 && b.w[nb - 1] == 0) nb--;
        if (na != nb) return na < nb ? -1 : 1;
        for (size_t i = na; i-- > 0;)
            if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
        return 0;
    }
};

// p^e > scale * p^(i w / 2), compared as p^(2e) > scale^2 p^(i w)
static bool exceeds(int p, int e, long long scale, int iw) {
    Big lhs, rhs;
    for (int k = 0; k < 2 * e; k++) lhs.mul(p);
    rhs.mul((uint64_t)scale);
    rhs.mul((uint64_t)scale);
    for (int k = 0; k < iw; k++) rhs.mul(p);
    return Big::cmp(lhs, rhs) > 0;
}

static long long binom_ll(int n, int k) { return binom(n, k); }

PrecOpts PrecOpts::from(const cr_family *fam) {
    PrecOpts o;
    o.r = fam->r;
    o.N = fam->n_series;
    for (int m = 0; m < kMaxVars; m++) o.Nm[m] = fam->n_series_m[m];
    o.M = fam->M;
    return o;
}

bool choose_precision(int p, int n, const std::vector<int> &hodge, const PrecOpts &o, int &r, std::vector<int> &Nm,
                      int &M, std::string &err) {
    std::vector<int> slopes;
    for (int m = 1; m <= n; m++)
        for (int k = 0; k < hodge[m - 1]; k++) slopes.push_back(n - m);
    std::sort(slopes.begin(), slopes.end());
    const int b = (int)slopes.size();
    const int w = n - 1;
    if (b == 0) {
        err = "empty cohomology basis";
        return false;
    }
    if (o.r < 0 || o.N < 0 || o.M < 0 || o.r > 64 || o.N > 64 || o.M > 128) {
        err = "precision override out of range";
        return false;
    }
    if (o.r > 0) {
        r = o.r;
    } else {
        r = 1;
        int mu = slopes[0], h = 0;
        for (int i = 1; i <= b / 2; i++) {
            h += slopes[i - 1];
            int rc = 1, rp = 1;
            while (!exceeds(p, rc + h, 2 * binom_ll(b, i), i * w)) rc++;
            while (!exceeds(p, rp + i * mu, 2LL * b, i * w)) rp++;
            r = std::max(r, std::min(rc, rp));
        }
    }
    const int N = o.N > 0 ? o.N : r + 1;
    Nm.assign(n, N);
    for (int m = 1; m <= n; m++) {
        if (o.Nm[m - 1] < 0 || o.Nm[m - 1] > 64) {
            err = "series order override out of range";
            return false;
        }
        if (o.Nm[m - 1] > 0) Nm[m - 1] = o.Nm[m - 1];
    }
    M = 0;
    for (int m = 1; m <= n; m++) {
        if (hodge[m - 1] == 0) continue;
        int sm = Nm[m - 1] + m - 1;
        M = std::max(M, r + vp_fact((long long)p * sm - 1, p) - m + 1);
    }
    if (o.M > 0) {
        if (o.M < M) {
            err = "working precision M = " + std::to_string(o.M) + " is below the " + std::to_string(M) +
                  " digits that keep r = " + std::to_string(r) + " digits in every column";
            return false;
        }
        M = o.M;
    }
    return true;
}

// Rank of an integer matrix mod a small prime (row-major rows x cols).
static int rank_mod_p(std::vector<int> a, int rows, int cols, int p) {
    int rank = 0;
    for (int c = 0; c < cols && rank < rows; c++) {
        int sel = -1;
        for (int r = rank; r < rows; r++)
            if (a[(size_t)r * cols + c] % p) {
                sel = r;
                break;
            }
        if (sel < 0) continue;
        if (sel != rank)
            for (int k = 0; k < cols; k++) std::swap(a[(size_t)sel * cols + k], a[(size_t)rank * cols + k]);
        int inv = 1;
        while ((a[(size_t)rank * cols + c] * inv) % p != 1) inv++;
        for (int k = 0; k < cols; k++) a[(size_t)rank * cols + k] = a[(size_t)rank * cols + k] * inv % p;
        for (int r = rank + 1; r < rows; r++) {
            int f = a[(size_t)r * cols + c] % p;
            if (!f) continue;
            for (int k = 0; k < cols; k++)
                a[(size_t)r * cols + k] = ((a[(size_t)r * cols + k] - f * a[(size_t)rank * cols + k]) % p + p) % p;
        }
        rank++;
    }
    return rank;
}

// Non-pivot columns of the row-echelon form mod p of a (rows x cols) matrix:
// column c is a pivot iff it is not a combination of columns 0..c-1.
static std::vector<int> nonpivot_columns_mod_p(std::vector<int> a, int rows, int cols, int p) {
    // Lazy reduction: a row below the pivots only accumulates g * (pivot row)
    // terms (g < p, pivot entries reduced below p), at most one per pivot,
    // so its entries stay below min(rows, cols) p^2 + p < 2^31 for the sizes
    // here and are reduced mod p only where they are tested or become a
    // pivot row.  The zero pattern mod p, and so the pivot columns, is that
    // of the reduced elimination.
    for (int &x : a) x = ((x % p) + p) % p;
    std::vector<int> out;
    int rank = 0;
    for (int c = 0; c < cols; c++) {
        int sel = -1;
        for (int r = rank; r < rows; r++)
            if (a[(size_t)r * cols + c] % p) {
                sel = r;
                break;
            }
        if (sel < 0) {
            out.push_back(c);
            continue;
        }
        if (sel != rank)
            for (int k = 0; k < cols; k++) std::swap(a[(size_t)sel * cols + k], a[(size_t)rank * cols + k]);
        int *pr = &a[(size_t)rank * cols];
        for (int k = c; k < cols; k++) pr[k] %= p;
        int inv = 1;
        while ((pr[c] * inv) % p != 1) inv++;
        for (int k = c; k < cols; k++) pr[k] = pr[k] * inv % p;
        for (int r = rank + 1; r < rows; r++) {
            int *ro = &a[(size_t)r * cols];
            const int f = ro[c] % p;
            if (!f) continue;
            const int g = p - f;  // ro - f pr = ro + (p - f) pr (mod p)
            for (int k = c; k < cols; k++) ro[k] += g * pr[k];
        }
        rank++;
    }
    return out;
}

// Right inverse of A (R x C, mod q): X (C x R) with A X = I.  Rows are taken in
// order; each row's pivot is its first column holding a unit after the
// earlier pivots were cleared.  Returns false if some row has no unit left
// (A is not surjective mod p).
//
// Left-looking form of that elimination: row r is brought up to date with
// the earlier pivot rows (in the state they had when they became pivots) in
// one pass, with the products summed in 128 bits and reduced once per 128
// terms (sparse pivot rows by their nonzero columns); the pivot rows are
// then cleared of the later pivot columns (back substitution, right half
// only).  The pivots, and so X, are those of
// plain Gauss-Jordan elimination in row order: the reduced rows are
// determined by the pivot columns.
static bool right_inverse(const ModQ &mq, int p, std::vector<u64> A, int R, int C, std::vector<u64> &X) {
    const int W = C + R;
    const u64 q = mq.q;
    std::vector<u64> a((size_t)R * W, 0);
    for (int r = 0; r < R; r++) {
        std::memcpy(&a[(size_t)r * W], &A[(size_t)r * C], sizeof(u64) * C);
        a[(size_t)r * W + C + r] = 1;
    }
    std::vector<int> piv(R, -1);
    std::vector<char> used(C, 0);
    std::vector<u128> acc(W);
    // nonzero columns of each pivot row when it is sparse (empty: dense)
    std::vector<std::vector<int>> nzc(R);
    auto index_row = [&](const u64 *P, int k0, std::vector<int> &out) {
        out.clear();
        int cnt = 0;
        for (int k = k0; k < W; k++) cnt += P[k] != 0;
        if (2 * cnt >= W - k0) return;
        for (int k = k0; k < W; k++)
            if (P[k]) out.push_back(k);
    };
    for (int r = 0; r < R; r++) {
        u64 *row = &a[(size_t)r * W];
        // apply the pivot rows in order, products summed in 128 bits: the
        // multiplier of pivot row j is the entry at c_j after pivots 0 .. j-1
        if (r > 0) {
            for (int k = 0; k < W; k++) acc[k] = row[k];
            for (int j = 0, n = 0; j < r; j++) {
                const int cj = piv[j];
                const u64 f = mq.reduce(acc[cj]);
                acc[cj] = f;
                if (!f) continue;
                const u64 m = q - f;
                const u64 *P = &a[(size_t)j * W];
                if (nzc[j].empty())
                    for (int k = 0; k < W; k++) acc[k] += (u128)m * P[k];
                else
                    for (int k : nzc[j]) acc[k] += (u128)m * P[k];
                if (++n == 128) {
                    for (int k = 0; k < W; k++) acc[k] = mq.reduce(acc[k]);
                    n = 0;
                }
            }
            for (int k = 0; k < W; k++) row[k] = mq.reduce(acc[k]);
        }
        int c = -1;
        for (int k = 0; k < C; k++)
            if (!used[k] && row[k] % (u64)p) {
                c = k;
                break;
            }
        if (c < 0) return false;
        const u64 inv = mq.inv(row[c]);
        for (int k = 0; k < W; k++)
            if (row[k]) row[k] = mq.mul(row[k], inv);
        used[c] = 1;
        piv[r] = c;
        index_row(row, 0, nzc[r]);
    }
    // back substitution on the right half: row r loses the later pivot
    // columns, row R - 1 first
    index_row(&a[(size_t)(R - 1) * W], C, nzc[R - 1]);
    for (int r = R - 2; r >= 0; r--) {
        u64 *row = &a[(size_t)r * W];
        bool any = false;
        for (int j = r + 1; j < R && !any; j++) any = row[piv[j]] != 0;
        if (any) {
            for (int k = C; k < W; k++) acc[k] = row[k];
            for (int j = r + 1, n = 0; j < R; j++) {
                const u64 f = row[piv[j]];
                if (!f) continue;
                const u64 m = q - f;
                const u64 *P = &a[(size_t)j * W];
                if (nzc[j].empty())
                    for (int k = C; k < W; k++) acc[k] += (u128)m * P[k];
                else
                    for (int k : nzc[j]) acc[k] += (u128)m * P[k];
                if (++n == 128) {
                    for (int k = C; k < W; k++) acc[k] = mq.reduce(acc[k]);
                    n = 0;
                }
            }
            for (int k = C; k < W; k++) row[k] = mq.reduce(acc[k]);
        }
        index_row(row, C, nzc[r]);
    }
    X.assign((size_t)C * R, 0);
    for (int r = 0; r < R; r++) std::memcpy(&X[(size_t)piv[r] * R], &a[(size_t)r * W + C], sizeof(u64) * R);
    return true;
}

// partial derivatives of f as dense polys over Homog_{d-1}
static std::vector<std::vector<long long>> derivatives(const Family &fam, const std::vector<long long> &f,
                                                       MonoSpace &dsp) {
    dsp.init(fam.nv, fam.d - 1);
    std::vector<std::vector<long long>> out(fam.nv, std::vector<long long>(dsp.count, 0));
    int e[kMaxVars];
    for (int k = 0; k < fam.coeff.count; k++) {
        if (!f[k]) continue;
        for (int i = 0; i < fam.nv; i++) {
            int ei = fam.coeff.at(k)[i];
            if (!ei) continue;
            for (int j = 0; j < fam.nv; j++) e[j] = fam.coeff.at(k)[j] - (j == i);
            out[i][dsp.rank(e)] += f[k] * ei;
        }
    }
    return out;
}

// Matrix of (mu_i) -> sum_i mu_i * base_i into Homog_k, base_i over Homog_{bdeg};
// multipliers of block i range over Homog_{k - bdeg}.  Row-major (dim Homog_k) x (columns).
static std::vector<long long> multiplier_matrix(const Family &fam, const std::vector<std::vector<long long>> &base,
                                                const MonoSpace &bsp, const MonoSpace &ksp,
                                                const std::vector<const MonoSpace *> &mult, int &ncols) {
    ncols = 0;
    for (auto *m : mult) ncols += m->count;
    std::vector<long long> A((size_t)ksp.count * ncols, 0);
    int e[kMaxVars];
    int col = 0;
    for (int i = 0; i < fam.nv; i++) {
        const MonoSpace &msp = *mult[i];
        for (int a = 0; a < msp.count; a++, col++)
            for (int t = 0; t < bsp.count; t++) {
                long long c = base[i][t];
                if (!c) continue;
                for (int j = 0; j < fam.nv; j++) e[j] = msp.at(a)[j] + bsp.at(t)[j];
                A[(size_t)ksp.rank(e) * ncols + col] += c;
            }
    }
    return A;
}

cr_status setup_item(const Family &fam, int p, const uint32_t *coeffs, const PrecOpts &prec, ItemSetup &out,
                     std::string &err, bool smooth_only, bool host_psi) {
    const int nv = fam.nv, n = fam.n, d = fam.d;
    if (!is_prime(p)) {
        err = "p is not prime";
        return CR_ENOTPRIME;
    }
    if (p < 7 || p >= 50 || p <= n || d % p == 0) {
        err = "need 7 <= p < 50, p > n, p not dividing d";
        return CR_EPRANGE;
    }
    std::vector<long long> f(fam.coeff.count);
    for (int k = 0; k < fam.coeff.count; k++) {
        if (coeffs[k] >= (uint32_t)p) {
            err = "coefficients must lie in [0, p)";
            return CR_EINVAL;
        }
        f[k] = coeffs[k];
    }
    out = ItemSetup();
    out.p = p;
    MonoSpace dsp;
    auto df = derivatives(fam, f, dsp);
    // x_i d_i f over Homog_d
    std::vector<std::vector<long long>> xdf(nv, std::vector<long long>(fam.coeff.count, 0));
    {
        int e[kMaxVars];
        for (int i = 0; i < nv; i++)
            for (int t = 0; t < dsp.count; t++) {
                if (!df[i][t]) continue;
                for (int j = 0; j < nv; j++) e[j] = dsp.at(t)[j] + (j == i);
                xdf[i][fam.coeff.rank(e)] += df[i][t];
            }
    }
    // smoothness: Jacobian criterion in degree (n+1)(d-2)+1 when S is not everything
    if (fam.nS != nv) {
        MonoSpace ksp, msp;
        ksp.init(nv, (n + 1) * (d - 2) + 1);
        msp.init(nv, (n + 1) * (d - 2) + 1 - (d - 1));
        std::vector<const MonoSpace *> mult(nv, &msp);
        int ncols;
        auto A = multiplier_matrix(fam, df, dsp, ksp, mult, ncols);
        std::vector<int> Ai(A.size());
        for (size_t k = 0; k < A.size(); k++) Ai[k] = (int)(A[k] % p);
        if (rank_mod_p(Ai, ksp.count, ncols, p) != ksp.count) {
            err = "f is singular mod p";
            return CR_ESINGULAR;
        }
    }
    // J_S into Homog_D: blocks d_i f (i in S) and x_i d_i f (i not in S)
    std::vector<std::vector<long long>> base(nv);
    for (int i = 0; i < nv; i++) base[i] = ((fam.smask >> i) & 1u) ? df[i] : xdf[i];
    // the two base spaces differ (Homog_{d-1} vs Homog_d); build block by block
    std::vector<long long> J((size_t)fam.tgt.count * fam.nsrc, 0);
    {
        int e[kMaxVars];
        for (int i = 0; i < nv; i++) {
            bool inS = (fam.smask >> i) & 1u;
            const MonoSpace &bsp = inS ? dsp : fam.coeff;
            const MonoSpace &msp = fam.srcblk[i];
            for (int a = 0; a < msp.count; a++)
                for (int t = 0; t < bsp.count; t++) {
                    long long c = base[i][t];
                    if (!c) continue;
                    for (int j = 0; j < nv; j++) e[j] = msp.at(a)[j] + bsp.at(t)[j];
                    J[(size_t)fam.tgt.rank(e) * fam.nsrc + fam.srcoff[i] + a] += c;
                }
        }
    }
    if (smooth_only) {
        std::vector<int> Ji(J.size());
        for (size_t k = 0; k < J.size(); k++) Ji[k] = (int)(J[k] % p);
        if (rank_mod_p(Ji, fam.tgt.count, fam.nsrc, p) != fam.tgt.count) {
            if (fam.nS == nv) {
                err = "f is singular mod p";
                return CR_ESINGULAR;
            }
            err = "f is not S-smooth";
            return CR_ENOT_S_SMOOTH;
        }
    }
    if (smooth_only) return CR_OK;
    // precision from the Hodge numbers of a smooth hypersurface of this degree
    // (the basis computed below must have exactly these sizes)
    std::vector<int> hodge_generic(n, 0);
    for (int m = 1; m <= n; m++) {
        const int k = d * m - n - 1;
        long long hsz = 0;
        for (int j = 0; j < nv; j++) {
            const int kk = k - j * (d - 1);
            if (kk < 0) break;
            hsz += ((j & 1) ? -1 : 1) * binom(nv, j) * count_monomials(nv, kk);
        }
        hodge_generic[m - 1] = (int)hsz;
    }
    if (!choose_precision(p, n, hodge_generic, prec, out.r, out.Nm, out.M, err)) return CR_EINVAL;
    {
        u128 q = 1;
        for (int k = 0; k < out.M; k++) {
            q *= (u64)p;
            if (q >> 55) {
                err = "p^M exceeds the 55-bit residues of this build";
                return CR_EPRECISION;
            }
        }
        out.mq.init((u64)q);
    }
    const ModQ &mq = out.mq;
    // psi = right inverse of J_S over Z/q (Proposition 3.3 decomposition); on
    // the device path k_psi builds J_S from the coefficients itself
    if (host_psi) {
        std::vector<u64> Jq(J.size());
        for (size_t k = 0; k < J.size(); k++) Jq[k] = mq.from_int(J[k]);
        std::vector<u64> X;
        if (!right_inverse(mq, p, Jq, fam.tgt.count, fam.nsrc, X)) {
            if (fam.nS == nv) {
                err = "f is singular mod p";
                return CR_ESINGULAR;
            }
            err = "f is not S-smooth";
            return CR_ENOT_S_SMOOTH;
        }
        out.psi.swap(X);
    }
    // basis B_m (Section 2.3)
    std::vector<std::vector<int>> Bm(n + 1);
    std::vector<MonoSpace> ksp(n + 1);
    out.hodge.assign(n, 0);
    for (int m = 1; m <= n; m++) {
        int k = d * m - n - 1;
        ksp[m].init(nv, k);
        if (ksp[m].count == 0) continue;
        MonoSpace msp;
        msp.init(nv, k - d + 1);
        std::vector<const MonoSpace *> mult(nv, &msp);
        int ncols;
        auto A = multiplier_matrix(fam, df, dsp, ksp[m], mult, ncols);
        // rows = generators, columns = monomials of Homog_k
        std::vector<int> G((size_t)ncols * ksp[m].count);
        for (int r = 0; r < ksp[m].count; r++)
            for (int c = 0; c < ncols; c++) G[(size_t)c * ksp[m].count + r] = (int)(A[(size_t)r * ncols + c] % p);
        Bm[m] = nonpivot_columns_mod_p(G, ncols, ksp[m].count, p);
        out.hodge[m - 1] = (int)Bm[m].size();
    }
    for (int m = 1; m <= n; m++)
        for (size_t k = 0; k < Bm[m].size(); k++) out.col_pole.push_back(m);
    out.b = (int)out.col_pole.size();
    if (out.hodge != hodge_generic) {
        err = "basis sizes differ from the Hodge numbers of a smooth hypersurface";
        return CR_ESINGULAR;
    }
    // rho: pole-n numerators -> basis coordinates (Section 3.3, step (2))
    {
        const int F = fam.fin.count, b = out.b;
        out.rho.assign((size_t)b * F, 0);
        std::vector<int> rowoff(n + 2, 0);
        for (int m = 1; m <= n; m++) rowoff[m + 1] = rowoff[m] + out.hodge[m - 1];
        // Pm: (dim Homog_k) x F, current map from pole-n numerators to pole-m numerators
        std::vector<u64> Pm((size_t)F * F, 0);
        for (int t = 0; t < F; t++) Pm[(size_t)t * F + t] = 1;
        for (int m = n; m >= 1; m--) {
            const MonoSpace &K = ksp[m];
            if (K.count == 0) break;
            MonoSpace msp;
            msp.init(nv, K.deg - d + 1);
            std::vector<const MonoSpace *> mult(nv, &msp);
            int ngen;
            auto A = multiplier_matrix(fam, df, dsp, K, mult, ngen);
            const int hm = out.hodge[m - 1], C = ngen + hm;
            std::vector<u64> Aq((size_t)K.count * C, 0);
            for (int r = 0; r < K.count; r++)
                for (int c = 0; c < ngen; c++) Aq[(size_t)r * C + c] = mq.from_int(A[(size_t)r * ngen + c]);
            for (int j = 0; j < hm; j++) Aq[(size_t)Bm[m][j] * C + ngen + j] = 1;
            std::vector<u64> X;
            if (!right_inverse(mq, p, Aq, K.count, C, X)) {
                err = "Griffiths-Dwork system not solvable";
                return CR_ESELFCHECK;
            }
            // at m = n, Pm is the identity on Homog_{dn-n-1} (K is that space)
            const bool ident = m == n && K.count == F;
            auto times_pm = [&](int row, int t) -> u64 {  // (X Pm)[row, t]
                if (ident) return X[(size_t)row * K.count + t];
                u128 acc = 0;
                for (int k = 0; k < K.count; k++) {
                    acc += (u128)X[(size_t)row * K.count + k] * Pm[(size_t)k * F + t];
                    if ((k & 127) == 127) acc = mq.reduce(acc);
                }
                return mq.reduce(acc);
            };
            // coordinates of B_m: rows ngen..ngen+hm-1 of X, composed with Pm
            for (int j = 0; j < hm; j++)
                for (int t = 0; t < F; t++) out.rho[(size_t)(rowoff[m] + j) * F + t] = times_pm(ngen + j, t);
            if (m == 1) break;
            // P_{m-1} = (m-1)^{-1} * Deriv * X[0..ngen) * Pm
            const MonoSpace &K2 = ksp[m - 1];
            std::vector<u64> AP((size_t)ngen * F, 0);
            for (int c = 0; c < ngen; c++)
                for (int t = 0; t < F; t++) AP[(size_t)c * F + t] = times_pm(c, t);
            std::vector<u64> Pn((size_t)std::max(K2.count, 1) * F, 0);
            u64 inv = mq.inv((u64)(m - 1));
            int e[kMaxVars];
            int c = 0;
            for (int i = 0; i < nv; i++)
                for (int a = 0; a < msp.count; a++, c++) {
                    int ei = msp.at(a)[i];
                    if (!ei) continue;
                    for (int j = 0; j < nv; j++) e[j] = msp.at(a)[j] - (j == i);
                    int row = K2.rank(e);
                    u64 w = mq.mul((u64)ei, inv);
                    for (int t = 0; t < F; t++)
                        Pn[(size_t)row * F + t] = mq.add(Pn[(size_t)row * F + t], mq.mul(w, AP[(size_t)c * F + t]));
                }
            Pm.swap(Pn);
        }
    }
    // Frobenius start terms (Proposition 2.1), grouped by the x^S-form exponent E'
    {
        const int b = out.b;
        int Nmax = 1;
        for (int m = 1; m <= n; m++) Nmax = std::max(Nmax, out.Nm[m - 1]);
        std::vector<MonoSpace> psp(Nmax);
        std::vector<std::vector<u64>> fpow(Nmax);
        psp[0].init(nv, 0);
        fpow[0].assign(1, 1);
        int e[kMaxVars];
        for (int j = 1; j < Nmax; j++) {
            psp[j].init(nv, d * j);
            fpow[j].assign(psp[j].count, 0);
            for (int a = 0; a < psp[j - 1].count; a++) {
                if (!fpow[j - 1][a]) continue;
                for (int k = 0; k < fam.coeff.count; k++) {
                    if (!f[k]) continue;
                    for (int i = 0; i < nv; i++) e[i] = psp[j - 1].at(a)[i] + fam.coeff.at(k)[i];
                    int idx = psp[j].rank(e);
                    fpow[j][idx] = mq.add(fpow[j][idx], mq.mul(fpow[j - 1][a], (u64)f[k]));
                }
            }
        }
        // E' = p (gamma + 1) - 1 + 1_S with gamma = beta + alpha of degree d L - n - 1,
        // L = m + j = P / p: one dense slot table per pole level, indexed by the
        // rank of gamma (ranks run in lexicographically descending order)
        int nlev = 1;
        for (int m = 1; m <= n; m++) nlev = std::max(nlev, m + out.Nm[m - 1] - 1);
        std::vector<MonoSpace> lsp(nlev + 1);
        std::vector<std::vector<int>> slot(nlev + 1);
        for (int L = 1; L <= nlev; L++) {
            lsp[L].init(nv, d * L - n - 1);
            slot[L].assign(lsp[L].count, -1);
        }
        std::vector<int> lev_of, rank_of;  // per distinct start term
        std::vector<u64> acc;              // nterm x b coefficients
        int col = 0;
        std::vector<u64> scale(Nmax);
        for (int m = 1; m <= n; m++) {
            const int N = out.Nm[m - 1], sm = N + m - 1;
            // scale_j = D_{j,m} (p s_m - 1)! / (p (m + j) - 1)!, the same for every column of pole m
            u64 ratio = 1;
            long long t = (long long)p * sm - 1;
            for (int j = N - 1; j >= 0; j--) {
                // D_{j,m} = (-1)^j sum_{i=j}^{N-1} C(m+i-1, i) C(i, j)
                i128 Dj = 0;
                for (int i = j; i < N; i++) Dj += (i128)binom(m + i - 1, i) * binom(i, j);
                if (j & 1) Dj = -Dj;
                i128 Dr = Dj % (i128)mq.q;
                if (Dr < 0) Dr += (i128)mq.q;
                for (; t >= (long long)p * (m + j); t--) ratio = mq.mul(ratio, (u64)t % mq.q);
                scale[j] = mq.mul((u64)Dr, ratio);
            }
            // scale_j f^j, shared by the columns of pole m
            std::vector<std::vector<u64>> sf(N);
            for (int j = 0; j < N; j++) {
                sf[j].resize(psp[j].count);
                for (int a = 0; a < psp[j].count; a++) sf[j][a] = fpow[j][a] ? mq.mul(scale[j], fpow[j][a]) : 0;
            }
            for (int bi = 0; bi < out.hodge[m - 1]; bi++, col++) {
                const int8_t *beta = ksp[m].at(Bm[m][bi]);
                for (int j = 0; j < N; j++) {
                    const int L = m + j;
                    for (int a = 0; a < psp[j].count; a++) {
                        if (!fpow[j][a]) continue;
                        for (int i = 0; i < nv; i++) e[i] = beta[i] + psp[j].at(a)[i];
                        const int rk = lsp[L].rank(e);
                        int &sl = slot[L][rk];
                        if (sl < 0) {
                            sl = (int)lev_of.size();
                            lev_of.push_back(L);
                            rank_of.push_back(rk);
                            acc.resize(acc.size() + b, 0);
                        }
                        u64 &v = acc[(size_t)sl * b + col];
                        v = mq.add(v, sf[j][a]);
                    }
                }
            }
        }
        // chains ordered by pole (descending), then exponent (descending), for balanced tiles
        const int gdeg = d * n - n;
        const size_t nterm = lev_of.size();
        std::vector<u64> &coef = out.coef;
        coef.assign(nterm * b, 0);
        out.chain_u.resize(nterm * nv);
        out.chain_g.resize(nterm);
        out.chain_pole.resize(nterm);
        size_t k = 0;
        for (int L = nlev; L >= 1; L--)
            for (int rk = 0; rk < lsp[L].count; rk++) {
                const int sl = slot[L][rk];
                if (sl < 0) continue;
                const int8_t *gmono = lsp[L].at(rk);
                // Algorithm 1 (Tweak): remove dn-n units from the front of E'
                int left = gdeg, gam[kMaxVars];
                for (int i = 0; i < nv; i++) {
                    const int E = p * (gmono[i] + 1) - 1 + (int)((fam.smask >> i) & 1u);
                    int take = std::min(E, left);
                    gam[i] = take;
                    out.chain_u[k * nv + i] = (int16_t)(E - take);
                    left -= take;
                }
                out.chain_g[k] = fam.g.rank(gam);
                if (out.chain_g[k] < 0) {
                    err = "start term outside Homog_{dn-n} after Tweak";
                    return CR_ESELFCHECK;
                }
                out.chain_pole[k] = p * L;
                std::memcpy(&coef[k * b], &acc[(size_t)sl * b], sizeof(u64) * b);
                out.column_steps += p * L - n;
                k++;
            }
    }
    // unscaling constants (Section 2.5): (p s_m - 1)!/(n-1)! = p^v * unit, per pole order m
    std::vector<int> vm(n + 1, 0);
    std::vector<u64> unitm(n + 1, 1);
    for (int m = 1; m <= n; m++) {
        const long long top = (long long)p * (out.Nm[m - 1] + m - 1) - 1;
        vm[m] = vp_fact(top, p);
        u64 unit = 1;
        for (long long t = n; t <= top; t++) {
            long long x = t;
            while (x % p == 0) x /= p;
            unit = mq.mul(unit, (u64)x % mq.q);
        }
        unitm[m] = unit;
    }
    for (int c = 0; c < out.b; c++) {
        const int m = out.col_pole[c];
        out.col_shift.push_back(vm[m] - (m - 1));
        out.col_prec.push_back(out.M - (vm[m] - (m - 1)));
        out.col_unit.push_back(unitm[m]);
    }
    return CR_OK;
}

// ------------------------------------------------------------------ digit representation
bool digit_params(int p, int M, int T, int nv, u64 wtmax, int dmax, DigitParams &dp) {
    int e = 1;
    while ((long long)std::llround(std::pow((double)p, e + 1)) <= 169) e++;
    const long long B = (long long)std::llround(std::pow((double)p, e));
    const int D = (M + e - 1) / e;
    if (D > dmax) return false;
    long double Q = 1;
    for (int k = 0; k < D; k++) Q *= B;
    if (Q >= std::ldexp(1.0L, 52)) return false;
    const long long half = (B - 1) / 2;
    // |S_k| <= D T half^2 (balanced digits on both sides), |Z_k| <= nv wtmax |S_k|
    const long double Smax = (long double)D * T * half * half;
    const long double Zmax = (long double)nv * (long double)wtmax * Smax;
    const long double lim = std::ldexp(1.0L, 53);
    auto span = [&](int a, int b) {  // Zmax * sum_{k=a}^{b-1} B^(k-a)
        long double acc = 0, pw = 1;
        for (int k = a; k < b; k++) {
            acc += pw;
            pw *= B;
        }
        return Zmax * acc;
    };
    // Horner split at h = D/2 (a constant of the kernel instance): both halves
    // must stay exact in fp64
    const int h = D / 2;
    if (!(span(h, D) < lim && span(0, h) < lim)) return false;
    // digit split: x in [0, Q') as x_hi B^ds + x_lo with both parts below 2^24
    const int ds = (D + 1) / 2;
    long double Bds = 1, Brest = 1;
    for (int k = 0; k < ds; k++) Bds *= B;
    for (int k = ds; k < D; k++) Brest *= B;
    if (Bds >= std::ldexp(1.0L, 24) || Brest >= std::ldexp(1.0L, 24)) return false;
    // floor division by B of v < 2^24: (mulhi(v, magic) >> shift) with
    // shift = floor(log2 B), magic = floor(2^(32 + shift) / B) + 1 < 2^32; exact
    // when B^2 < 2^(8 + shift) (error v (magic B - 2^(32+shift)) / 2^(32+shift) < 1/B)
    int ell = 0;
    while ((2LL << ell) <= B) ell++;
    if ((long long)B * B >= (1LL << (8 + ell))) return false;
    dp.e = e;
    dp.B = (int)B;
    dp.D = D;
    dp.h = h;
    dp.ds = ds;
    dp.halfB = (int)half;
    // Z32: the weighted sums z_k and the carry sums t_k = z_k + c_k fit int32
    // (|c_(k+1)| <= |t_k| / B + 1/2, so |t_k| <= (Zmax + 1/2) B / (B - 1))
    dp.z32 = (Zmax + 0.5L) * (long double)B / (long double)(B - 1) < std::ldexp(1.0L, 31) - 1 ? 1 : 0;
    dp.shift = ell;
    dp.magic = (uint32_t)(((1ULL << (32 + ell)) / (unsigned long long)B) + 1);
    dp.Qp = (u64)Q;
    dp.Bd = (double)B;
    dp.Qd = (double)dp.Qp;
    dp.invQ = 1.0 / dp.Qd;
    long double BH = 1, Bh = 1, bias = 0, pw = 1;
    for (int k = 0; k < D - h; k++) BH *= B;
    for (int k = 0; k < h; k++) Bh *= B;
    for (int k = 0; k < D; k++) {
        bias += half * pw;
        pw *= B;
    }
    dp.BHd = (double)BH;
    dp.invBH = 1.0 / dp.BHd;
    dp.Bh = (double)Bh;
    dp.Bsplit = (double)Bds;
    dp.invBsplit = 1.0 / dp.Bsplit;
    dp.bias = (double)bias;
    return true;
}

bool bin_layout(const Family &fam, int nrt, BinLayout &bl) {
    const int s = fam.g.count, nv = fam.nv;
    struct Group {
        int r;
        std::vector<int> members;  // variable index i of each source row
    };
    std::vector<Group> groups;
    int maxsz = 0;
    for (int r = 0; r < s; r++) {
        Group g{r, {}};
        for (int i = 0; i < nv; i++)
            if (fam.gsrc[(size_t)r * nv + i] >= 0) g.members.push_back(i);
        if (!g.members.empty()) {
            maxsz = std::max(maxsz, (int)g.members.size());
            groups.push_back(g);
        }
    }
    if (maxsz > 4) return false;
    bl.nbins = 2 * nrt;
    // Every bin gets the kernel instance's constant pattern of group slots:
    // three-row groups (variables 0, 1, 2 in order) in the three-row slots,
    // one-row groups of variable z in the one-row slots reserved for z, spread
    // round-robin over the bins.  Anything else falls back to another kernel.
    const int ng = slot_groups(nrt);
    if (ng == 0 || nv != 3) return false;
    struct Slot {
        int bin, start, size, var;
        bool used;
    };
    std::vector<Slot> slots;
    {
        int start = 0;
        for (int g = 0; g < ng; g++) {
            for (int b = 0; b < bl.nbins; b++) slots.push_back({b, start, slot_group(nrt, g), slot_var(nrt, g), false});
            start += slot_group(nrt, g);
        }
        if (start > 16) return false;
    }
    bl.slot_src.assign((size_t)bl.nbins * 16, -1);
    bl.slot.assign((size_t)bl.nbins * 16, 0);
    for (const Group &g : groups) {
        const int sz = (int)g.members.size();
        const bool full = sz == 3 && g.members[0] == 0 && g.members[1] == 1 && g.members[2] == 2;
        if (!full && sz != 1) return false;
        Slot *pick = nullptr;
        for (auto &sl : slots)
            if (!sl.used && sl.size == sz && (full || sl.var == g.members[0])) {
                pick = &sl;
                break;
            }
        if (!pick) return false;
        pick->used = true;
        for (int m = 0; m < sz; m++) {
            const int i = g.members[m], j = pick->start + m;
            const int src = fam.gsrc[(size_t)g.r * nv + i];
            const int gwv = fam.gw[(size_t)g.r * nv + i];
            bl.slot_src[(size_t)pick->bin * 16 + j] = src;
            bl.slot[(size_t)pick->bin * 16 + j] = 1u | ((m == sz - 1) ? 2u : 0u) | ((uint32_t)i << 2) |
                                                  ((uint32_t)gwv << 5) | ((uint32_t)g.r << 16);
        }
    }
    // unused group slots still mark their end, so every lane runs the same code
    for (auto &sl : slots)
        if (!sl.used) bl.slot[(size_t)sl.bin * 16 + sl.start + sl.size - 1] |= 2u | (0xFFFFu << 16);
    return true;
}

bool quad_layout(const Family &fam, int nrt, int nrtf, BinLayout &bl) {
    const int s = fam.g.count, nv = fam.nv;
    if (nv != 4 || fam.nS != 4) return false;
    bl.nbins = 2 * nrt;
    bl.slot_src.assign((size_t)bl.nbins * 16, -1);
    bl.slot.assign((size_t)bl.nbins * 16, 0);
    // quads in accumulator order: full row tiles first (one output with all
    // four sources per quad), then single row tiles (slot t: a one-source
    // output of variable t)
    int full_q = 0;
    std::vector<int> single_q(nv, 0);
    const int full_cap = nrtf * 2 * 4, single_cap = (nrt - nrtf) * 2 * 4;
    for (int r = 0; r < s; r++) {
        int members[4], cnt = 0;
        for (int i = 0; i < nv; i++)
            if (fam.gsrc[(size_t)r * nv + i] >= 0) members[cnt++] = i;
        if (cnt == 0) continue;
        if (cnt != 4 && cnt != 1) return false;
        int qd, bin;
        if (cnt == 4) {
            if (full_q >= full_cap) return false;
            qd = full_q++;
            bin = qd / 4;
        } else {
            const int z = members[0];
            if (single_q[z] >= single_cap) return false;
            qd = single_q[z]++;
            bin = 2 * nrtf + qd / 4;
        }
        for (int m = 0; m < cnt; m++) {
            const int i = members[m], j = (qd % 4) * 4 + i;  // slot t of the quad is variable t
            bl.slot_src[(size_t)bin * 16 + j] = fam.gsrc[(size_t)r * nv + i];
            bl.slot[(size_t)bin * 16 + j] =
                1u | ((uint32_t)i << 2) | ((uint32_t)fam.gw[(size_t)r * nv + i] << 5) | ((uint32_t)r << 16);
        }
    }
    // every quad of a full row tile is a whole group or empty (marked r = 0xFFFF)
    for (int qd = full_q; qd < full_cap; qd++) bl.slot[(size_t)(qd / 4) * 16 + (qd % 4) * 4] = 0xFFFFu << 16;
    return true;
}

bool wide_layout(const Family &fam, int nrt, int nrtq, BinLayout &bl) {
    const int s = fam.g.count, nv = fam.nv;
    if (nv != 5 || nrtq > nrt) return false;
    bl.nbins = 2 * nrt;
    bl.slot_src.assign((size_t)bl.nbins * 16, -1);
    bl.slot.assign((size_t)bl.nbins * 16, 0);
    const int five_cap = nrtq * 2 * 3, single_cap = nrtq * 2 + (nrt - nrtq) * 2 * 16;
    int nfive = 0, nsingle = 0;
    for (int r = 0; r < s; r++) {
        int members[5], cnt = 0;
        for (int i = 0; i < nv; i++)
            if (fam.gsrc[(size_t)r * nv + i] >= 0) members[cnt++] = i;
        if (cnt == 0) continue;
        int bin, j0;
        if (cnt == 5) {
            if (nfive >= five_cap) return false;
            bin = nfive / 3;
            j0 = (nfive % 3) * 5;
            nfive++;
        } else if (cnt == 1) {
            if (nsingle >= single_cap) return false;
            if (nsingle < nrtq * 2) {
                bin = nsingle;
                j0 = 15;
            } else {
                const int t = nsingle - nrtq * 2;
                bin = 2 * nrtq + t / 16;
                j0 = t % 16;
            }
            nsingle++;
        } else {
            return false;
        }
        for (int m = 0; m < cnt; m++) {
            const int i = members[m], j = cnt == 5 ? j0 + i : j0;  // five-source slot 5 q + i is variable i
            bl.slot_src[(size_t)bin * 16 + j] = fam.gsrc[(size_t)r * nv + i];
            bl.slot[(size_t)bin * 16 + j] =
                1u | ((uint32_t)i << 2) | ((uint32_t)fam.gw[(size_t)r * nv + i] << 5) | ((uint32_t)r << 16);
        }
    }
    // an unused five-source group is marked r = 0xFFFF in its first slot
    for (int q = nfive; q < five_cap; q++) bl.slot[(size_t)(q / 3) * 16 + (q % 3) * 5] = 0xFFFFu << 16;
    return true;
}

bool quad_digit_params(int p, int M, int T, int nv, u64 wtmax, DigitParams &dp) {
    int e = 1;
    while ((long long)std::llround(std::pow((double)p, e + 1)) <= 169) e++;
    const long long B = (long long)std::llround(std::pow((double)p, e));
    const int D = (M + e - 1) / e;
    long double Q = 1;
    for (int k = 0; k < D; k++) Q *= B;
    if (Q >= std::ldexp(1.0L, 52)) return false;
    const long long half = (B - 1) / 2;
    // int32 MFMA accumulation: |Z_k| <= D T half^2
    const long double Smax = (long double)D * T * half * half;
    if (Smax >= std::ldexp(1.0L, 31) - 1) return false;
    // weighted sums and carry sums: |t_k| <= (nv wtmax Smax + 1/2) B / (B - 1) < 2^48
    const long double tmax = ((long double)nv * (long double)wtmax * Smax + 0.5L) * B / (long double)(B - 1);
    if (tmax >= std::ldexp(1.0L, 48)) return false;
    dp = DigitParams();
    // int32 finish: accumulators within 24-bit multiplies and the carry sums within int32
    dp.z32 = Smax < std::ldexp(1.0L, 23) - 1 && tmax < std::ldexp(1.0L, 31) - 1 ? 1 : 0;
    dp.e = e;
    dp.B = (int)B;
    dp.D = D;
    dp.halfB = (int)half;
    dp.Qp = (u64)Q;
    dp.Bd = (double)B;
    dp.Qd = (double)dp.Qp;
    dp.invQ = 1.0 / dp.Qd;
    return true;
}

void pack_psi_digits(const Family &fam, const ItemSetup &it, const DigitParams &dp, int nrt, int nkb, int8_t *out,
                     const BinLayout *bl) {
    const int D = dp.D, T = fam.tgt.count, half = (dp.B - 1) / 2;
    const long long B = dp.B;
    const u64 Q = dp.Qp, bias = (Q - 1) / 2;
    std::vector<int8_t> dig((size_t)fam.nsrc * T * D);
    // x / B as the high product with ceil(2^64 / B): it never undershoots and
    // overshoots by at most one for x < 2^52, which the remainder test corrects
    const u64 rB = ~0ull / (u64)B + 1;
    for (size_t e = 0; e < (size_t)fam.nsrc * T; e++) {
        // balanced digits of x = unsigned digits of (x + (Q-1)/2) mod Q, minus (B-1)/2
        u64 x = it.psi[e] + bias;
        if (x >= Q) x -= Q;
        for (int i = 0; i < D; i++) {
            u64 qd = (u64)(((u128)x * rB) >> 64);
            if (qd * (u64)B > x) qd--;
            dig[e * D + i] = (int8_t)((int)(x - qd * (u64)B) - half);
            x = qd;
        }
    }
    for (int rt = 0; rt < nrt; rt++)
        for (int i = 0; i < D; i++)
            for (int kb = 0; kb < nkb; kb++)
                for (int lane = 0; lane < 64; lane++) {
                    int row = 32 * rt + lane % 32;
                    if (bl) {  // MFMA row 32 rt + rho holds source row slot_src[bin][slot]
                        const int rho = lane % 32, h = (rho >> 2) & 1, j = (rho >> 3) * 4 + (rho & 3);
                        row = bl->slot_src[(size_t)(2 * rt + h) * 16 + j];
                        if (row < 0) row = fam.nsrc;  // padding: zero row
                    }
                    const int k0 = 32 * kb + (lane / 32) * 16;
                    int8_t *dst = out + ((((size_t)rt * D + i) * nkb + kb) * 64 + lane) * 16;
                    for (int j = 0; j < 16; j++) {
                        const int k = k0 + j;
                        dst[j] = (row < fam.nsrc && k < T) ? dig[((size_t)row * T + k) * D + i] : 0;
                    }
                }
}

// ------------------------------------------------------------------ chunk counter
void count_chunks(const Family &fam, const int16_t *u0, int pole, int64_t &chunks) {
    int U[kMaxVars], v[kMaxVars];
    for (int i = 0; i < fam.nv; i++) U[i] = u0[i];
    while (pole > fam.n) {
        int left = fam.d;
        for (int i = 0; i < fam.nv; i++) v[i] = 0;
        for (int s = 0; s < fam.nv && left > 0; s++)
            if (((fam.smask >> s) & 1u) && U[s]) {
                v[s] = 1;
                left--;
            }
        while (left > 0) {
            bool moved = false;
            for (int m = 0; m < fam.nv && left > 0; m++)
                if (v[m] < U[m]) {
                    v[m]++;
                    left--;
                    moved = true;
                }
            if (!moved) return;
        }
        int k = pole - fam.n;
        for (int i = 0; i < fam.nv; i++)
            if (v[i]) k = std::min(k, U[i] / v[i]);
        for (int i = 0; i < fam.nv; i++) U[i] -= k * v[i];
        pole -= k;
        chunks++;
    }
}

// ------------------------------------------------------------------ finishing
// Characteristic polynomial det(I - T A) mod Q by Berkowitz's division-free
// recursion: for A = [[a, R], [C, A1]], chi_A = Toeplitz(1, -a, -RC, -RA1C, ...) chi_A1.
static std::vector<u64> charpoly_mod(const ModQ &mq, const std::vector<u64> &A, int b) {
    std::vector<u64> poly{1, mq.sub(0, A[(size_t)(b - 1) * b + (b - 1)])};
    for (int k = b - 2; k >= 0; k--) {
        const int m = b - k;  // size of the current trailing block
        std::vector<u64> t(m + 1, 0);
        t[0] = 1;
        t[1] = mq.sub(0, A[(size_t)k * b + k]);
        std::vector<u64> vcur(m - 1), vnext(m - 1);
        for (int i = 0; i < m - 1; i++) vcur[i] = A[(size_t)(k + 1 + i) * b + k];  // C
        for (int j = 2; j <= m; j++) {
            u128 acc = 0;
            for (int i = 0; i < m - 1; i++) acc += (u128)A[(size_t)k * b + k + 1 + i] * vcur[i] % mq.q;
            t[j] = mq.sub(0, (u64)(acc % mq.q));
            if (j == m) break;
            for (int i = 0; i < m - 1; i++) {
                u128 s = 0;
                for (int l = 0; l < m - 1; l++) s += (u128)A[(size_t)(k + 1 + i) * b + k + 1 + l] * vcur[l] % mq.q;
                vnext[i] = (u64)(s % mq.q);
            }
            vcur.swap(vnext);
        }
        std::vector<u64> np(m + 1, 0);
        for (int i = 0; i <= m; i++) {
            u128 acc = 0;
            for (int j = 0; j < (int)poly.size() && j <= i; j++) acc += (u128)t[i - j] * poly[j] % mq.q;
            np[i] = (u64)(acc % mq.q);
        }
        poly.swap(np);
    }
    return poly;
}

static i128 symlift(u64 x, u64 Q) { return (2 * (u128)x > Q) ? (i128)x - (i128)Q : (i128)x; }

static bool mul_ok(i128 a, i128 b, i128 &out) { return !__builtin_mul_overflow(a, b, &out); }

static u64 ipow(u64 p, int e) {
    u64 r = 1;
    while (e-- > 0) r *= p;
    return r;
}

cr_status finish_item(const Family &fam, const ItemSetup &it, const u64 *Y, u64 *frob, int32_t *col_pole,
                      int32_t *col_prec, int64_t *lpoly, std::string &err) {
    const int b = it.b, p = it.p, n = fam.n, w = n - 1;
    std::vector<u64> phi((size_t)b * b);
    for (int c = 0; c < b; c++) {
        const u64 div = ipow(p, it.col_shift[c]);
        const u64 Qc = ipow(p, it.col_prec[c]);
        ModQ mc;
        mc.init(Qc);
        const u64 uinv = mc.inv(it.col_unit[c] % Qc);
        for (int i = 0; i < b; i++) {
            u64 y = Y[(size_t)i * b + c];
            if (y % div) {
                err = "Frobenius column not divisible by the expected power of p";
                return CR_ESELFCHECK;
            }
            phi[(size_t)i * b + c] = mc.mul((y / div) % Qc, uinv);
        }
        col_pole[c] = it.col_pole[c];
        col_prec[c] = it.col_prec[c];
    }
    std::memcpy(frob, phi.data(), sizeof(u64) * b * b);
    // ---- Q(T): a_i for i <= b/2 from the Weil bound, the rest from the functional equation
    std::vector<int> slope(b);
    for (int c = 0; c < b; c++) slope[c] = n - it.col_pole[c];
    std::vector<int> sorted = slope;
    std::sort(sorted.begin(), sorted.end());
    const int mu = sorted[0], r = it.r, half = b / 2;
    std::vector<int> use_coef(half + 1, 0);
    int K1 = 0, K2 = 0, h = 0;
    for (int i = 1; i <= half; i++) {
        h += sorted[i - 1];
        if (exceeds(p, r + h, 2 * binom(b, i), i * w)) {
            use_coef[i] = 1;
            K1 = std::max(K1, r + h);
        } else if (exceeds(p, r + i * mu, 2LL * b, i * w)) {
            K2 = std::max(K2, r + i * mu);
        } else {
            err = "precision too small to recover Q(T)";
            return CR_EPRECISION;
        }
    }
    auto fits = [&](int K) { return K <= 0 || (double)K * __builtin_log2((double)p) < 62.0; };
    if (!fits(K1) || !fits(K2)) {
        err = "Q(T) recovery modulus exceeds 64 bits";
        return CR_EPRECISION;
    }
    std::vector<u64> cpoly, psum;
    if (K1 > 0) {
        ModQ m1;
        m1.init(ipow(p, K1));
        std::vector<u64> A((size_t)b * b);
        for (int i = 0; i < b; i++)
            for (int c = 0; c < b; c++) A[(size_t)i * b + c] = m1.mul(phi[(size_t)i * b + c] % m1.q, ipow(p, slope[c]) % m1.q);
        cpoly = charpoly_mod(m1, A, b);
    }
    if (K2 > 0) {
        ModQ m2;
        m2.init(ipow(p, K2));
        std::vector<u64> A((size_t)b * b), P((size_t)b * b, 0), T((size_t)b * b);
        for (int i = 0; i < b; i++)
            for (int c = 0; c < b; c++) A[(size_t)i * b + c] = m2.mul(phi[(size_t)i * b + c] % m2.q, ipow(p, slope[c]) % m2.q);
        for (int i = 0; i < b; i++) P[(size_t)i * b + i] = 1;
        for (int k = 1; k <= half; k++) {
            for (int i = 0; i < b; i++)
                for (int j = 0; j < b; j++) {
                    u128 acc = 0;
                    for (int l = 0; l < b; l++) acc += (u128)P[(size_t)i * b + l] * A[(size_t)l * b + j] % m2.q;
                    T[(size_t)i * b + j] = (u64)(acc % m2.q);
                }
            P.swap(T);
            u64 tr = 0;
            for (int i = 0; i < b; i++) tr = m2.add(tr, P[(size_t)i * b + i]);
            psum.push_back(tr);
        }
    }
    std::vector<i128> a(b + 1, 0), s;
    a[0] = 1;
    for (int i = 1; i <= half; i++) {
        if (use_coef[i]) {
            int hi = 0;
            for (int k = 0; k < i; k++) hi += sorted[k];
            a[i] = symlift(cpoly[i] % ipow(p, r + hi), ipow(p, r + hi));
            i128 si = -(i128)i * a[i];
            for (int k = 1; k < i; k++) {
                i128 t;
                if (!mul_ok(s[k - 1], a[i - k], t)) goto overflow;
                si -= t;
            }
            s.push_back(si);
        } else {
            const u64 Q2 = ipow(p, r + i * mu);
            i128 si = symlift(psum[i - 1] % Q2, Q2);
            s.push_back(si);
            i128 num = 0;
            for (int k = 1; k <= i; k++) {
                i128 t;
                if (!mul_ok(s[k - 1], a[i - k], t)) goto overflow;
                num -= t;
            }
            if (num % i) {
                err = "Newton identity not integral";
                return CR_ESELFCHECK;
            }
            a[i] = num / i;
        }
    }
    {
        // sign: det(Phi') mod p must be +-1
        ModQ mp;
        mp.init((u64)p);
        std::vector<u64> M((size_t)b * b);
        for (size_t k = 0; k < M.size(); k++) M[k] = phi[k] % p;
        u64 det = 1;
        for (int c = 0; c < b; c++) {
            int sel = -1;
            for (int r2 = c; r2 < b; r2++)
                if (M[(size_t)r2 * b + c]) {
                    sel = r2;
                    break;
                }
            if (sel < 0) {
                det = 0;
                break;
            }
            if (sel != c) {
                for (int k = 0; k < b; k++) std::swap(M[(size_t)sel * b + k], M[(size_t)c * b + k]);
                det = mp.sub(0, det);
            }
            det = mp.mul(det, M[(size_t)c * b + c]);
            u64 inv = mp.inv(M[(size_t)c * b + c]);
            for (int r2 = c + 1; r2 < b; r2++) {
                u64 f = mp.mul(M[(size_t)r2 * b + c], inv);
                if (!f) continue;
                for (int k = c; k < b; k++) M[(size_t)r2 * b + k] = mp.sub(M[(size_t)r2 * b + k], mp.mul(f, M[(size_t)c * b + k]));
            }
        }
        int eps;
        if (det == 1) eps = 1;
        else if (det == (u64)p - 1) eps = -1;
        else {
            err = "det Phi' is not +-1 mod p";
            return CR_ESELFCHECK;
        }
        const int sgn = ((b & 1) ? -1 : 1) * eps;
        for (int i = 0; i < (b + 1) / 2; i++) {
            const int e2 = w * (b - 2 * i);
            i128 pw = 1, t;
            for (int k = 0; k < e2 / 2; k++)
                if (!mul_ok(pw, (i128)p, pw)) goto overflow;
            if (!mul_ok(pw, a[i], t)) goto overflow;
            a[b - i] = sgn * t;
        }
        if (b % 2 == 0 && sgn == -1 && a[b / 2] != 0) {
            err = "functional equation violated";
            return CR_ESELFCHECK;
        }
    }
    for (int i = 0; i <= b; i++) {
        u128 x = (u128)a[i];
        uint64_t fill = a[i] < 0 ? ~0ull : 0ull;
        lpoly[4 * i + 0] = (int64_t)(uint64_t)x;
        lpoly[4 * i + 1] = (int64_t)(uint64_t)(x >> 64);
        lpoly[4 * i + 2] = (int64_t)fill;
        lpoly[4 * i + 3] = (int64_t)fill;
    }
    return CR_OK;
overflow:
    err = "Q(T) coefficients exceed 127 bits";
    return CR_EPRECISION;
}

}  // namespace crf
