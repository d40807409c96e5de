// Host-side setup and finishing of the controlled-reduction pipeline.
//
// Everything here runs once per hypersurface (setup) or once per family
// (index tables); the per-step work runs in the HIP kernels of kernels.hip.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/crfrob.h"

namespace crf {

using u64 = uint64_t;
using u128 = unsigned __int128;
using i128 = __int128;

constexpr int kMaxVars = 6;

// ---------------------------------------------------------------- modulus
// Residues mod q = p^M, q < 2^55.  Barrett reduction of x < 2^(2*sbits+8):
//   qhat = ((x >> (sbits-1)) * mu) >> (sbits+9),  mu = floor(2^(2*sbits+8) / q),
// then at most two corrective subtractions.  The device uses the same formula
// with the constants computed here.
struct ModQ {
    u64 q = 0;
    int sbits = 0;
    u64 mu = 0;
    void init(u64 modulus);
    u64 reduce(u128 x) const {
        if (sbits > 55) return (u64)(x % q);  // only the small finishing moduli exceed the Barrett range
        u64 x1 = (u64)(x >> (sbits - 1));
        u64 qh = (u64)(((u128)x1 * mu) >> (sbits + 9));
        u64 r = (u64)x - qh * q;
        while (r >= q) r -= q;
        return r;
    }
    u64 mul(u64 a, u64 b) const { return reduce((u128)a * b); }
    u64 add(u64 a, u64 b) const { u64 s = a + b; return s >= q ? s - q : s; }
    u64 sub(u64 a, u64 b) const { return a >= b ? a - b : a + q - b; }
    u64 inv(u64 a) const;  // a must be a unit
    u64 from_int(long long v) const {
        long long r = v % (long long)q;
        return (u64)(r < 0 ? r + (long long)q : r);
    }
};

// ---------------------------------------------------------------- monomials
// Homogeneous monomials of one degree in nv variables, lex-descending.
// rank() maps an exponent vector to its position by counting the monomials
// that precede it (combinatorial number system).
struct MonoSpace {
    int nv = 0, deg = -1, count = 0;
    std::vector<int8_t> exps;  // count x nv
    void init(int nvars, int degree);
    int rank(const int *e) const;  // -1 if e has a negative entry or wrong degree
    const int8_t *at(int k) const { return exps.data() + (size_t)k * nv; }
};

long long binom(int n, int k);
long long count_monomials(int nv, int deg);

// ---------------------------------------------------------------- family
// Index tables that depend only on (nvars, degree, S).
struct Family {
    int nv = 0, n = 0, d = 0, nS = 0;
    uint32_t smask = 0;  // bit i set <=> i in S
    int D = 0;           // degree of the J_S target: dn + d - n - |S|
    MonoSpace coeff;     // Homog_d          (input coefficients)
    MonoSpace g;         // Homog_{dn-n}     (s: numerators g of Proposition 3.3)
    MonoSpace tgt;       // Homog_D          (x^v g / x^S)
    MonoSpace fin;       // Homog_{dn-n-1}   (pole-n numerators)
    MonoSpace dirs;      // Homog_d          (directions v, |v| = d)
    std::vector<MonoSpace> srcblk;  // block i: Homog_{D-d+1} (i in S) or Homog_{D-d}
    std::vector<int> srcoff;        // offsets of the blocks, size nv+1
    int nsrc = 0;
    // colmap[dir*s + k] = tgt rank of v_dir + g_k - 1_S, or -1
    std::vector<int16_t> colmap;
    // gather for R_{u,v}: for output monomial r (g-space) and variable i,
    // gsrc = src index of r - 1_S + [i in S] e_i (or -1), gw = r_i + [i not in S]
    std::vector<int16_t> gsrc, gw;
    // final exponents U (|U| = |S| - 1) and finmap[Uidx*s + k] = fin rank of U + g_k - 1_S or -1
    MonoSpace finU;
    std::vector<int16_t> finmap;
    // J_S from the coefficients of f: entry (t, srcoff[i] + a) is the
    // coefficient c_e of f times w, jtab = (e << 8) | w, or -1 when it is 0
    // (x^beta, beta = tgt_t - srcblk_i[a], is a monomial of d_i f (i in S:
    // e = rank(beta + e_i), w = beta_i + 1) or of x_i d_i f (e = rank(beta),
    // w = beta_i))
    std::vector<int32_t> jtab;  // tgt.count x nsrc
    bool init(int nvars, int degree, uint32_t s_mask, std::string &err);
};

// ---------------------------------------------------------------- per item
struct ItemSetup {
    int p = 0, r = 0, M = 0, b = 0;
    std::vector<int> Nm;             // series order N_m, m = 1..n (index m-1)
    ModQ mq;
    std::vector<int> hodge;          // |B_m|, m = 1..n (index m-1)
    std::vector<int> col_pole;       // b
    std::vector<u64> psi;            // nsrc x T, right inverse of J_S mod q (host_psi)
    std::vector<u64> rho;            // b x F, Griffiths-Dwork coordinates of pole-n numerators
    // start blocks (one chain each), sorted by pole descending
    std::vector<int16_t> chain_u;    // nchain x nv
    std::vector<int32_t> chain_g;    // g-space rank of the Tweak remainder
    std::vector<int32_t> chain_pole; // pole order P
    std::vector<u64> coef;           // nchain x b
    std::vector<int> col_shift;      // v_p((p s_m - 1)!) - (m - 1)
    std::vector<int> col_prec;       // M - col_shift
    std::vector<u64> col_unit;       // unit part of (p s_m - 1)!/(n-1)! mod q
    int64_t column_steps = 0, chunks = 0;
    std::vector<int8_t> apack;       // psi digits for the MFMA kernel (empty if unused)
    int nchain() const { return (int)chain_g.size(); }
};

// Caller overrides of the precision parameters of Section 2.5 (cr_family).
struct PrecOpts {
    int r = 0;              // relative precision; 0 = derive
    int N = 0;              // N_m for every m; 0 = r + 1
    int Nm[kMaxVars] = {};  // N_m of pole order m = 1..n (index m-1); 0 = N
    int M = 0;              // working precision; 0 = the least that keeps r digits in every column
    static PrecOpts from(const cr_family *fam);
};

// Precision of Section 2.5 under the reading in crfrob.h: r, N_m (m = 1..n)
// and M.  Fails (err set) if an override is out of range or M is below the
// least working precision for r.
bool choose_precision(int p, int n, const std::vector<int> &hodge, const PrecOpts &o, int &r, std::vector<int> &Nm,
                      int &M, std::string &err);

// S-smoothness test + full setup of one item.  Returns CR_OK or an error status.
// With host_psi false the right inverse of J_S is not computed: out.J holds
// J_S mod q for the device (k_psi), and a non-surjective J_S is reported there.
cr_status setup_item(const Family &fam, int p, const uint32_t *coeffs, const PrecOpts &prec, ItemSetup &out,
                     std::string &err, bool smooth_only = false, bool host_psi = true);

// Unscale the device result Y (b x b mod q) and recover Q(T).
cr_status finish_item(const Family &fam, const ItemSetup &it, const u64 *Y, u64 *frob,
                      int32_t *col_pole, int32_t *col_prec, int64_t *lpoly, std::string &err);

// Parameters of the int8-digit representation of Z/Q' used by the MFMA kernel
// (Q' = B^D, B = p^e <= 255 odd, balanced digits; see kernels_mfma.hip).
struct DigitParams {
    int e = 0, B = 0, D = 0, h = 0, ds = 0, halfB = 0, z32 = 0, shift = 0;
    uint32_t magic = 0;
    u64 Qp = 0;
    double Bd = 0, Qd = 0, invQ = 0, BHd = 0, invBH = 0, Bh = 0, Bsplit = 0, invBsplit = 0, bias = 0;
};
// Chooses B, D and the Horner split h so that every recombination is exact in
// fp64 and the weighted gather fits in 64 bits.  Returns false if no choice does.
bool digit_params(int p, int M, int T, int nv, u64 wtmax, int dmax, DigitParams &dp);
// Placement of the J_S source rows in the MFMA accumulator layout so that every
// output r of the weighted gather finds all its source rows src(r, i) in ONE
// lane.  Lane half h of wave w holds rows 32 w + (j/4)*8 + h*4 + (j%4),
// j = 0..15 ("bin" 2 w + h, "slot" j).  Each source row feeds exactly one
// output (r -> r - 1_S + [i in S] e_i is injective), so the rows are
// partitioned into groups, one per output, packed whole into bins.
struct BinLayout {
    int nbins = 0;
    std::vector<int> slot_src;    // nbins x 16: source row or -1
    std::vector<uint32_t> slot;   // nbins x 16: packed (valid | end << 1 | i << 2 | gw << 5 | r << 16)
};
bool bin_layout(const Family &fam, int nrt, BinLayout &bl);

// Row placement of the four-variable quad kernel (S = all): nrt row tiles, the
// first nrtf of them full quads (the four source rows of one output, slot t =
// variable t), the others single quads (four one-source outputs, slot t of
// variable t); slot words as in BinLayout (end bit unused, r = 0xFFFF marks
// an empty full quad).  False if the family's groups do not fit.
bool quad_layout(const Family &fam, int nrt, int nrtf, BinLayout &bl);

// Row placement of the streaming kernel for cubic threefolds (five variables, S = {x_4}):
// nrt row tiles, the first nrtq of them "quint" tiles whose lane halves hold
// three five-source outputs (slots 5 q + i: variable i) and one one-source
// output (slot 15), the others sixteen one-source outputs per lane half; slot
// words as in BinLayout (bits 2-4 the variable, r = 0xFFFF marks an empty
// five-source group).  False if the family's outputs do not fit.
bool wide_layout(const Family &fam, int nrt, int nrtq, BinLayout &bl);
// Digits of the quad and streaming kernels: B = p^e <= 169, D = ceil(M / e),
// Q' = B^D < 2^52, int32 position sums, carry sums below 2^48; z32 set when
// the position sums fit 24-bit multiplies and the carry sums int32.
bool quad_digit_params(int p, int M, int T, int nv, u64 wtmax, DigitParams &dp);

// psi digits in v_mfma_i32_32x32x32_i8 A-fragment order:
// out[(((rt*D + i)*nkb + kb)*64 + lane)*16 + j] = digit i of psi[32 rt + lane%32][32 kb + (lane/32)*16 + j]
void pack_psi_digits(const Family &fam, const ItemSetup &it, const DigitParams &dp, int nrt, int nkb, int8_t *out,
                     const BinLayout *bl = nullptr);

// Depth-first chunk schedule statistics of one chain (host mirror of the device
// policy, used for counters only).
void count_chunks(const Family &fam, const int16_t *u0, int pole, int64_t &chunks);

}  // namespace crf
