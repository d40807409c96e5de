// Device-side data layout shared by the C-ABI host code and the HIP kernels.
#pragma once
#include <cstdint>

namespace crf {

// Per-family index tables (depend on nvars, degree and S only).
struct DevFamily {
    int nv, n, d;
    uint32_t smask;
    int s;      // dim Homog_{dn-n}: length of the reduced vectors g
    int T;      // dim Homog_D: target of J_S
    int nsrc;   // sum of the J_S source blocks
    int F;      // dim Homog_{dn-n-1}: pole-n numerators
    int ndir;   // directions v with |v| = d
    int nfinU;  // final exponents U with |U| = |S| - 1
    const int16_t *colmap;  // ndir x s : tgt index of v + g_k - 1_S (or -1)
    const int16_t *gsrc;    // s x nv   : src index of r - 1_S + [i in S] e_i (or -1)
    const int16_t *gw;      // s x nv   : r_i + [i not in S]
    const int16_t *finmap;  // nfinU x s: fin index of U + g_k - 1_S (or -1)
    const int8_t *dirs;     // ndir x nv
    const int8_t *finU;     // nfinU x nv
};

// Per-hypersurface data.
struct DevItem {
    uint64_t q;      // p^M
    uint64_t mu;     // Barrett constant floor(2^(2 sbits + 8) / q)
    int32_t sbits;   // bit length of q (<= 55)
    int32_t b;       // side of Phi'
    int32_t chain0;  // first chain (global index)
    int32_t nchain;
    int32_t nfin;    // vectors that reach pole n
    int32_t p;
    const uint64_t *psi;   // nsrc x T right inverse of J_S
    const uint64_t *rho;   // b x F Griffiths-Dwork coordinate map
    const uint64_t *coef;  // (nchain + b) x b: start coefficients, then the unit rows e_c
    const int32_t *fvec;   // nfin: global index of each vector that reaches pole n
    const int32_t *frow;   // nfin: its coefficient row in coef
    uint64_t *Y;           // b x b output (coordinates, mod q)
    uint64_t *H;           // F x b scratch: summed pole-n numerators
    const uint32_t *fcoef; // coefficients of f (input of k_psi, which builds J_S from them)
    uint64_t *psi_out;     // the psi buffer above, written by k_psi
    int32_t *flag;         // set by k_psi when J_S has no unit pivot in some row
};

// Per reduced vector (one entry per vector of every phase of a plan).
struct DevVec {
    int32_t pend;  // pole at which the vector stops
    int32_t in;    // store row holding the start vector, or -1: the unit vector e_gamma
    int32_t out;   // store row receiving the result, or -1: pole-n numerators (hbuf row)
    int32_t dir;   // direction forced for the whole range, or -1: Algorithm 3 chunks
};

// A store row built between two phases: row = sum_{m0 <= j < m1} alpha_j src_j
// (src_j >= 0 a store row, src_j < 0 the unit vector e_{-src_j - 1}).
struct DevComb {
    int32_t row, item, m0, m1;
};

// A tile of chains of one item processed by one workgroup.
struct DevTile {
    int32_t item;
    int32_t chain0;  // global index of the first chain
    int32_t count;
    int32_t steps;   // longest chain of the tile (pole - n)
};

}  // namespace crf

namespace crf {

// Digit (p-adic) representation used by the MFMA reduction kernel.  Residues
// live in Z/Q', Q' = B^D with B = p^e <= 169 (a multiple-power of p at least
// p^M), as D balanced base-B digits (|digit| <= (B-1)/2, stored as int8).
// Products of digits at positions >= D are multiples of Q' and are dropped.
struct DevDigitItem {
    double Bd;            // base B
    double Qd, invQ;      // Q' = B^D
    double BHd, invBH;    // B^(D-h)
    double Bh;            // B^h
    double Bsplit, invBsplit;  // B^ds: the digit split cuts x into x_hi * B^ds + x_lo
    double bias;          // sum_j halfB B^j when digits are balanced, else 0
    uint64_t Qp;          // Q'
    uint64_t q;           // p^M (final reduction)
    uint32_t magic;       // floor division by B of a value < 2^24: mulhi(v, magic) >> shift
    int32_t shift;
    int32_t B;
    int32_t halfB;        // subtracted from every digit when balanced, else 0
    int32_t D;            // digits
    int32_t h;            // Horner split position
    int32_t ds;           // digit split position
    int32_t z32;          // 1: the weighted digit sums and the carry sums fit int32
    int32_t fold;         // 1: psi digits packed for the tile-pair kernel (folded last K-block)
    int32_t chain0, nchain;
    const int8_t *apack;  // NRT x D x NKB x 64 lanes x 16 bytes: psi digits in MFMA A-fragment order
    int8_t *apack_out;    // the same buffer, written by k_pack_psi
};

}  // namespace crf

namespace crf {

// Lane-slot pattern of the register-gather kernel: the output groups held by
// one lane bin, the same in every bin (a group is the set of source rows
// src(r, i) that feed output r, stored at the group's slots in the order of
// i).  For S = all variables in three variables a group has all three
// variables (r_i >= 1 for every i) or exactly one, the variable z with
// r_z = 0.  Each one-row slot position is reserved for one variable, so the
// variable of every slot is a constant of the pattern; empty slots hold
// zero rows of psi and contribute nothing.  Quartic curves (2 row tiles,
// 4 bins, two one-row slots per variable) and quintic curves (4 row tiles,
// 8 bins, one per variable).
constexpr int kSlotGroups2[] = {3, 3, 3, 1, 1, 1, 1, 1, 1};
constexpr int kSlotVars2[] = {-1, -1, -1, 0, 1, 2, 0, 1, 2};
constexpr int kSlotGroups4[] = {3, 3, 3, 1, 1, 1};
constexpr int kSlotVars4[] = {-1, -1, -1, 0, 1, 2};
constexpr int slot_groups(int nrt) { return nrt == 2 ? 9 : (nrt == 4 ? 6 : 0); }
constexpr int slot_group(int nrt, int g) { return nrt == 2 ? kSlotGroups2[g] : kSlotGroups4[g]; }
// variable of a one-row group (-1 for a three-row group: variables 0, 1, 2 in order)
constexpr int slot_var(int nrt, int g) { return nrt == 2 ? kSlotVars2[g] : kSlotVars4[g]; }

}  // namespace crf
