// Exact int8-digit MFMA reduction for four-variable families with S = all
// variables (quartic K3 surfaces: s = 220, J_S with 336 source and 220 target
// rows).
//
// One step of a vector w at exponent u with direction v (Proposition 3.3 and
// the explicit R_{u,v} of Section 3.1):
//   t  = psi[:, cols(v)] w                          (nsrc values)
//   w'[r] = sum_i (u_i + r_i) t[src(r, i)]          (s values)
// For 32 vectors of one hypersurface, t is one integer product on the matrix
// cores: the vectors are scattered into the J_S target space (row v + g - 1),
// so vectors of different directions share it.  Residues live in Z/Q',
// Q' = B^D, B = p^e <= 169 odd, as D balanced int8 digits; the digit-position
// sums Z_k = sum_{i+j=k} psi_i X_j accumulate exactly in int32
// (v_mfma_i32_32x32x32_i8) and positions >= D, multiples of Q', are never
// formed.
//
// Shapes that differ from the plane-curve kernels: psi has 11 row tiles of 32
// and 7 K-blocks, too many digits to stay in registers, so each wave streams
// the digits of its row tiles from memory (L2) for every step, one row tile
// at a time, and finishes that row tile before the next one.  The gather runs
// on the accumulators: every output r has either all four source rows
// src(r, i) (r_i >= 1 for every i) or exactly one (r_z = 0 for one z), or
// none, and the host places the rows so that a lane's aligned quad of
// accumulator rows (rows 8 q + 4 h + t, t = 0..3, of lane half h) holds the
// four rows of one output ("full" row tiles) or four one-row outputs of
// variables 0, 1, 2, 3 ("single" row tiles).  Slot t of a quad is always
// variable t.
//
// The new digits come from carry propagation over the weighted position sums
// z_k: t = z_k + carry, carry = round(t / B), digit = t - B carry.  |t| stays
// below 2^48 (checked on the host), where t / B lies at least 1/(2B) from a
// half-integer (B odd) and the fp64 product t * (1/B) is within
// |t| 2^-52 / B of it, so rint gives the exact quotient.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_layout.hpp"

namespace crf {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kQV = 32;      // vectors per tile: the column tile of one MFMA
constexpr int kQWaves = 4;   // waves per workgroup, one per SIMD
constexpr int kQTab = 8192;  // colmap entries (ndir x s) held in LDS
constexpr int kQSmall = 256; // bytes for the direction and final-exponent tables

template <int NRT, int NKB, int D>
struct QuadShape {
    static constexpr int K = NKB * 32;
    static constexpr int XS = K + 16;          // bytes per (digit, vector) row of the planes
    static constexpr int XB = D * kQV * XS;    // one set of digit planes
    static constexpr size_t lds = 2 * (size_t)XB + kQTab * 2 + 2 * kQSmall + (size_t)NRT * 2 * 16 * 4;
};

// Algorithm 3 with S = all variables (greedy v: one unit on every variable
// with u_i != 0, then round robin while v_i < u_i) and the largest chunk k
// with u - k v >= 0, capped by the remaining pole orders; dir = index of v in
// the family's direction table (-1 if v is not complete).
__device__ __forceinline__ void choose_chunk_q(int d, int ndir, const int8_t *dirsL, const int *U, int poles_left,
                                               int *v, int &dir, int &k) {
    int left = d;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        v[i] = (left > 0 && U[i] != 0) ? 1 : 0;
        left -= v[i];
    }
    for (int guard = 0; guard < 64 && left > 0; guard++) {
        bool moved = false;
#pragma unroll
        for (int m = 0; m < 4; m++)
            if (left > 0 && v[m] < U[m]) {
                v[m]++;
                left--;
                moved = true;
            }
        if (!moved) break;
    }
    k = poles_left;
#pragma unroll
    for (int i = 0; i < 4; i++)
        if (v[i]) k = min(k, U[i] / v[i]);
    dir = -1;
    if (left == 0)
        for (int t = 0; t < ndir && dir < 0; t++)
            if (dirsL[4 * t] == v[0] && dirsL[4 * t + 1] == v[1] && dirsL[4 * t + 2] == v[2] && dirsL[4 * t + 3] == v[3])
                dir = t;
}

// A fragments (psi digits 0..D-1) of row tile rt, K-block kb; base = the
// item's packed digits plus this lane's 16-byte offset.
// The loads go through a global-address-space pointer: as generic (flat)
// loads they would also count on the LDS counter, and every wait for the
// digit planes would then wait for the prefetch as well.
typedef const __attribute__((address_space(1))) v4i gv4i;

template <int D, int NKB>
__device__ __forceinline__ void load_frags(const int8_t *base, int rt, int kb, v4i (&dst)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) dst[i] = *(gv4i *)(base + (((size_t)rt * D + i) * NKB + kb) * 1024);
}

// Fragments of digit planes 0..D-1 of K-block kb (LDS); xc = this lane's
// vector row plus its 16-byte half.
template <int D, int XS>
__device__ __forceinline__ void load_planes(const int8_t *xc, int kb, v4i (&dst)[D]) {
#pragma unroll
    for (int j = 0; j < D; j++) dst[j] = *reinterpret_cast<const v4i *>(xc + (size_t)j * kQV * XS + kb * 32);
}

// Balanced base-B digits of x in [0, q) (q | Q'), written D planes apart.
// v < Q' < 2^52 is exact in fp64: the quotient by B from the product with
// 1 / B is off by at most one, which the remainder's range corrects (a 64-bit
// integer division costs far more).
template <int D, int XS>
__device__ __forceinline__ void put_digits_q(int8_t *xp, uint64_t x, uint64_t Qp, int B, double invB, int halfB) {
    uint64_t v = x + (Qp - 1) / 2;  // unsigned digits of x + sum_k halfB B^k, mod Q'
    if (v >= Qp) v -= Qp;
#pragma unroll
    for (int k = 0; k < D; k++) {
        uint64_t qd = (uint64_t)((double)v * invB);
        int64_t r = (int64_t)(v - qd * (uint64_t)B);
        if (r < 0) {
            qd--;
            r += B;
        } else if (r >= B) {
            qd++;
            r -= B;
        }
        xp[k * kQV * XS] = (int8_t)((int)r - halfB);
        v = qd;
    }
}

// Output r of vector c from its balanced digits dg[0..D-1] (the carry
// propagation over its weighted position sums): either the digits of the
// next step or the final value mod q (combine store or pole-n numerators).
template <int D, int XS>
__device__ __forceinline__ void put_out_q(const int (&dg)[D], int r, bool more, const int16_t *cm, int8_t *Xn_c,
                                          int vout, int fin_row, const int16_t *__restrict__ finmap, uint64_t *hrow,
                                          uint64_t *__restrict__ store, int s, int64_t Bi, int64_t q, int &bad) {
    if (more) {
        const int col = cm[r];
        if (col < 0) {
            bool nz = false;
#pragma unroll
            for (int k = 0; k < D; k++) nz = nz || dg[k] != 0;
            if (nz) bad |= 2;
            return;
        }
#pragma unroll
        for (int k = 0; k < D; k++) Xn_c[k * kQV * XS + col] = (int8_t)dg[k];
        return;
    }
    int64_t x = 0;
#pragma unroll
    for (int k = D - 1; k >= 0; k--) x = x * Bi + dg[k];
    // x mod q for |x| < Q' / 2 < 2^51 (exact in fp64): the floored quotient
    // from the product with 1 / q is off by at most one
    x -= (int64_t)floor((double)x * (1.0 / (double)q)) * q;
    if (x < 0) x += q;
    else if (x >= q) x -= q;
    if (x == 0) return;  // outputs were cleared at the start of the tile
    if (vout >= 0) {
        store[(size_t)vout * s + r] = (uint64_t)x;
    } else if (fin_row >= 0) {
        const int f = finmap[fin_row + r];
        if (f < 0) bad |= 4;
        else hrow[f] = (uint64_t)x;
    }
}

// Four outputs of this lane half of a row tile: their weighted position
// sums z_k, then their carry propagations side by side, position by position
// (four independent chains in flight instead of one), then their digits out.
// FULL: the row tile's four full quads, one output each (quad o, its rows
// 4 o + t with weights of variable t); else the four one-row outputs of
// single quad qd (row 4 qd + t, variable t).
//
// Z32 (the host has bounded |acc| < 2^23 and |t_k| < 2^31 for the item): the
// sums are 24-bit multiply-adds in int32 and carry = round(t / B) is the low
// word of t / B + 1.5 2^52 in fp64 (for |t| < 2^31 the product's error, below
// 2^-22, cannot carry t / B across a half-integer, which it lies at least
// 1 / (2B) from); the digit t - B carry is only needed mod 2^8 (|d| < 128),
// where a 24-bit multiply-add gives it.  Otherwise fp64 throughout: |t_k| <
// 2^48 (checked on the host) keeps t * (1/B) within |t| 2^-52 / B of t / B,
// so rint gives the exact quotient.
template <int D, int XS, bool FULL, bool Z32>
__device__ __forceinline__ void finish4(const v16i (&acc)[D], int qd, const uint32_t *sb, const int (&up)[4],
                                        bool more, const int16_t *cm, int8_t *Xn_c, int vout, int fin_row,
                                        const int16_t *__restrict__ finmap, uint64_t *hrow,
                                        uint64_t *__restrict__ store, int s, double Bd, double invB, int Bs,
                                        int64_t Bi, int64_t q, int &bad) {
    int wt[4][4];
    int rr[4];
    bool ok[4];
#pragma unroll
    for (int o = 0; o < 4; o++) {
        if (FULL) {
            rr[o] = (int)(sb[4 * o] >> 16);
            ok[o] = rr[o] != 0xFFFF;
#pragma unroll
            for (int t = 0; t < 4; t++) wt[o][t] = up[t] + (int)((sb[4 * o + t] >> 5) & 2047u);
        } else {
            const uint32_t w = sb[4 * qd + o];
            rr[o] = (int)(w >> 16);
            ok[o] = (w & 1u) != 0;
            wt[o][0] = up[o] + (int)((w >> 5) & 2047u);
        }
    }
    int dg[4][D];
    if constexpr (Z32) {
        constexpr double kRound = 6755399441055744.0;  // 1.5 2^52
        int ci[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < D; k++)
#pragma unroll
            for (int o = 0; o < 4; o++) {
                int t = ci[o];
                if (FULL) {
#pragma unroll
                    for (int m = 0; m < 4; m++) t = __mul24(wt[o][m], acc[k][4 * o + m]) + t;
                } else {
                    t = __mul24(wt[o][0], acc[k][4 * qd + o]) + t;
                }
                ci[o] = __double2loint(fma((double)t, invB, kRound));
                // low 24 bits of the carry times 2^24 - B, plus t: = d_k mod 2^8
                unsigned du;
                asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(du) : "v"(ci[o]), "v"((1u << 24) - (unsigned)Bs), "v"(t));
                dg[o][k] = (int)(int8_t)(du & 0xffu);
            }
    } else {
        double z[4][D];
#pragma unroll
        for (int o = 0; o < 4; o++) {
#pragma unroll
            for (int k = 0; k < D; k++) z[o][k] = 0.0;
            if (FULL) {
#pragma unroll
                for (int m = 0; m < 4; m++)
#pragma unroll
                    for (int k = 0; k < D; k++) z[o][k] = fma((double)wt[o][m], (double)acc[k][4 * o + m], z[o][k]);
            } else {
#pragma unroll
                for (int k = 0; k < D; k++) z[o][k] = (double)wt[o][0] * (double)acc[k][4 * qd + o];
            }
        }
        double carry[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < D; k++)
#pragma unroll
            for (int o = 0; o < 4; o++) {
                const double v = z[o][k] + carry[o];
                const double cq = rint(v * invB);
                dg[o][k] = (int)fma(-cq, Bd, v);
                carry[o] = cq;
            }
    }
    // the carry out of position D - 1 is a multiple of Q' and is dropped.
    // The digits are pinned here: the compiler would otherwise sink each
    // output's whole chain into the branch that writes it, one chain after
    // the other again.
#pragma unroll
    for (int o = 0; o < 4; o++)
#pragma unroll
        for (int k = 0; k < D; k++) asm volatile("" : "+v"(dg[o][k]));
#pragma unroll
    for (int o = 0; o < 4; o++)
        if (ok[o]) put_out_q<D, XS>(dg[o], rr[o], more, cm, Xn_c, vout, fin_row, finmap, hrow, store, s, Bi, q, bad);
}

template <int NRT, int NRTF, int NKB, int D, bool Z32>
__device__ __forceinline__ void quad_tile(const DevFamily &fam, const DevTile &tile, const DevDigitItem *__restrict__ items,
                          const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
                          const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx,
                          uint64_t *__restrict__ store, uint64_t *__restrict__ hbuf, int &bad, int8_t *Xbuf,
                          const int16_t *colmapL, const int8_t *dirsL, const int8_t *finUL, const uint32_t *slotL) {
    using Sh = QuadShape<NRT, NKB, D>;
    constexpr int XS = Sh::XS, XB = Sh::XB, NT = 64 * kQWaves;
    const int s = fam.s, F = fam.F;
    const DevDigitItem it = items[tile.item];
    // the wave index is uniform over the wave: in a scalar register, every
    // row-tile offset below is scalar arithmetic
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int c = lane & 31, half = lane >> 5;
    const int nch = tile.count;

    for (int idx = tid; idx < 2 * XB / 16; idx += NT) reinterpret_cast<v4i *>(Xbuf)[idx] = v4i{0, 0, 0, 0};
    for (int idx = tid; idx < nch * F; idx += NT)
        if (vx[tile.chain0 + idx / F].out < 0) hbuf[(size_t)tile.chain0 * F + idx] = 0;
    for (int idx = tid; idx < nch * s; idx += NT) {
        const int out = vx[tile.chain0 + idx / s].out;
        if (out >= 0) store[(size_t)out * s + idx % s] = 0;
    }
    __syncthreads();

    const double Bd = it.Bd, invB = 1.0 / it.Bd;
    const int64_t Bi = it.B, q = (int64_t)it.q;

    // vector state (registers; identical in every lane of vector c)
    int U[4] = {0, 0, 0, 0}, V[4] = {0, 0, 0, 0};
    int dir = 0, kleft = 0, pole = fam.n, pend = fam.n, vout = -1;
    if (c < nch) {
        const int g = tile.chain0 + c;
        const DevVec xv = vx[g];
#pragma unroll
        for (int i = 0; i < 4; i++) U[i] = cu[(size_t)g * 4 + i];
        pole = cpole[g];
        pend = xv.pend;
        vout = xv.out;
        int d0, k0;
        if (xv.dir >= 0) {  // one forced direction for the whole range
            d0 = xv.dir;
            k0 = pole - pend;
#pragma unroll
            for (int i = 0; i < 4; i++) V[i] = dirsL[d0 * 4 + i];
        } else {
            choose_chunk_q(fam.d, fam.ndir, dirsL, U, pole - pend, V, d0, k0);
        }
        if (d0 < 0 || k0 < 1) {
            bad |= 1;
            d0 = 0;
            pole = pend;
        }
        dir = d0;
        kleft = k0;
        if (xv.in < 0) {
            if (wave == 0 && half == 0) {
                const int col = colmapL[d0 * s + cg[g]];
                if (col < 0) bad |= 2;
                else Xbuf[c * XS + col] = (int8_t)1;  // balanced digits of 1
            }
        } else {
            // start vector from the combine store: the 8 lanes of vector c split its entries
            for (int r = 2 * wave + half; r < s; r += 2 * kQWaves) {
                const uint64_t x = store[(size_t)xv.in * s + r];
                if (x == 0) continue;
                const int col = colmapL[d0 * s + r];
                if (col < 0) {
                    bad |= 2;
                    continue;
                }
                put_digits_q<D, XS>(Xbuf + c * XS + col, x, it.Qp, it.B, invB, it.halfB);
            }
        }
    }
    __syncthreads();

    int cur = 0;
    for (int step = 0; step < tile.steps; step++) {
        const int8_t *Xc = Xbuf + cur * XB;
        int8_t *Xn = Xbuf + (cur ^ 1) * XB;
        // bookkeeping of this lane's vector: exponent after the step, next direction
        const bool act = pole > pend;
        int up[4], Vn[4], dirn = dir, kleftn = kleft - 1;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            up[i] = U[i] - (act ? V[i] : 0);
            Vn[i] = V[i];
        }
        const bool more = act && pole - 1 > pend;
        if (more && kleftn == 0) {
            int d0, k0;
            choose_chunk_q(fam.d, fam.ndir, dirsL, up, pole - 1 - pend, Vn, d0, k0);
            if (d0 < 0 || k0 < 1) {
                bad |= 1;
                d0 = 0;
                k0 = 1 << 30;
            }
            dirn = d0;
            kleftn = k0;
        }
        int fin_row = -1;
        if (act && !more && vout < 0) {
            int Ui = -1;
            for (int a = 0; a < fam.nfinU && Ui < 0; a++)
                if (finUL[4 * a] == up[0] && finUL[4 * a + 1] == up[1] && finUL[4 * a + 2] == up[2] &&
                    finUL[4 * a + 3] == up[3])
                    Ui = a;
            if (Ui < 0) bad |= 4;
            else fin_row = Ui * s;
        }
        const int16_t *cm = colmapL + dirn * s;
        int8_t *Xn_c = Xn + c * XS;
        uint64_t *hrow = hbuf + (size_t)(tile.chain0 + c) * F;

        // psi digit fragments (L2) and plane fragments (LDS) one K-block ahead,
        // and the next row tile's first psi block during the last block and
        // the finish: one wave per SIMD has no other wave to hide the latency
        // of the loads.  The scheduling fences keep each block's loads ahead
        // of its products; without them the compiler sinks the loads to their
        // uses under register pressure, and every fragment waits for its load.
        const int8_t *abase = it.apack + lane * 16;
        const int8_t *xbase = Xc + c * XS + half * 16;
        v4i an[D], xn[D];
        if (wave < NRT) load_frags<D, NKB>(abase, wave, 0, an);
        for (int rt = wave; rt < NRT; rt += kQWaves) {
            v16i acc[D];
#pragma unroll
            for (int k = 0; k < D; k++) acc[k] = v16i{0};
            load_planes<D, XS>(xbase, 0, xn);
#pragma unroll
            for (int kb = 0; kb < NKB; kb++) {
                v4i xb[D], a[D];
#pragma unroll
                for (int i = 0; i < D; i++) {
                    a[i] = an[i];
                    xb[i] = xn[i];
                }
                if (kb + 1 < NKB) {
                    load_frags<D, NKB>(abase, rt, kb + 1, an);
                    load_planes<D, XS>(xbase, kb + 1, xn);
                } else if (rt + kQWaves < NRT) {
                    load_frags<D, NKB>(abase, rt + kQWaves, 0, an);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < D; i++)
#pragma unroll
                    for (int j = 0; i + j < D; j++)
                        acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], xb[j], acc[i + j], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (!act) continue;
            const uint32_t *sb = slotL + (rt * 2 + half) * 16;
            if (rt < NRTF) {
                // full quads: one output each, sources of variables 0..3 in slots 0..3
                finish4<D, XS, true, Z32>(acc, 0, sb, up, more, cm, Xn_c, vout, fin_row, fam.finmap, hrow, store, s,
                                          Bd, invB, it.B, Bi, q, bad);
            } else {
                // single quads: four one-row outputs, slot t of variable t
#pragma unroll
                for (int qd = 0; qd < 4; qd++)
                    finish4<D, XS, false, Z32>(acc, qd, sb, up, more, cm, Xn_c, vout, fin_row, fam.finmap, hrow,
                                               store, s, Bd, invB, it.B, Bi, q, bad);
            }
        }
        __syncthreads();  // every wave has read the current planes and written the next ones
        int8_t *Xz = Xbuf + cur * XB;
        for (int idx = tid; idx < XB / 16; idx += NT) reinterpret_cast<v4i *>(Xz)[idx] = v4i{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            U[i] = up[i];
            V[i] = Vn[i];
        }
        if (act) {
            pole -= 1;
            dir = dirn;
            kleft = kleftn;
        }
        cur ^= 1;
        __syncthreads();  // the cleared planes are free for the next step's digits
    }
}

// One tile with the digit count of its item, DLO or DHI, and its finish
// arithmetic, int32 where the item's bounds allow it (the hypersurfaces of
// one call may have different primes, hence different digit counts; one
// launch takes the tiles of all of them).
template <int NRT, int NRTF, int NKB, int DLO, int DHI>
__device__ __forceinline__ void quad_tile_any(const DevFamily &fam, const DevTile &tile,
                                              const DevDigitItem *__restrict__ items, const int16_t *__restrict__ cu,
                                              const int32_t *__restrict__ cg, const int32_t *__restrict__ cpole,
                                              const DevVec *__restrict__ vx, uint64_t *__restrict__ store,
                                              uint64_t *__restrict__ hbuf, int &bad, int8_t *Xbuf,
                                              const int16_t *colmapL, const int8_t *dirsL, const int8_t *finUL,
                                              const uint32_t *slotL) {
    const int D = __builtin_amdgcn_readfirstlane(items[tile.item].D);
    const int z32 = __builtin_amdgcn_readfirstlane(items[tile.item].z32);
    if (D == DLO) {
        if (z32)
            quad_tile<NRT, NRTF, NKB, DLO, true>(fam, tile, items, cu, cg, cpole, vx, store, hbuf, bad, Xbuf, colmapL,
                                                 dirsL, finUL, slotL);
        else
            quad_tile<NRT, NRTF, NKB, DLO, false>(fam, tile, items, cu, cg, cpole, vx, store, hbuf, bad, Xbuf, colmapL,
                                                  dirsL, finUL, slotL);
    } else {
        if (z32)
            quad_tile<NRT, NRTF, NKB, DHI, true>(fam, tile, items, cu, cg, cpole, vx, store, hbuf, bad, Xbuf, colmapL,
                                                 dirsL, finUL, slotL);
        else
            quad_tile<NRT, NRTF, NKB, DHI, false>(fam, tile, items, cu, cg, cpole, vx, store, hbuf, bad, Xbuf, colmapL,
                                                  dirsL, finUL, slotL);
    }
}

// One workgroup per tile (queue == nullptr) or a persistent grid draining the
// tile list through the counter *queue (zero at launch; every workgroup
// leaves once the counter passes ntiles).  The LDS is laid out for DHI.
template <int NRT, int NRTF, int NKB, int DLO, int DHI>
__global__ __launch_bounds__(64 * kQWaves) void k_reduce_quad(
    DevFamily fam, const DevDigitItem *__restrict__ items, const DevTile *__restrict__ tiles, int ntiles,
    int *__restrict__ queue, const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
    const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx, uint64_t *__restrict__ store,
    uint64_t *__restrict__ hbuf, const uint32_t *__restrict__ slots, int *__restrict__ err) {
    using Sh = QuadShape<NRT, NKB, DHI>;
    extern __shared__ __align__(16) unsigned char ldsq[];
    int8_t *Xbuf = reinterpret_cast<int8_t *>(ldsq);
    int16_t *colmapL = reinterpret_cast<int16_t *>(ldsq + 2 * (size_t)Sh::XB);
    int8_t *dirsL = reinterpret_cast<int8_t *>(colmapL + kQTab);
    int8_t *finUL = dirsL + kQSmall;
    uint32_t *slotL = reinterpret_cast<uint32_t *>(finUL + kQSmall);
    __shared__ int next;
    const int NT = 64 * kQWaves, tid = threadIdx.x;
    for (int idx = tid; idx < fam.ndir * fam.s; idx += NT) colmapL[idx] = fam.colmap[idx];
    for (int idx = tid; idx < fam.ndir * 4; idx += NT) dirsL[idx] = fam.dirs[idx];
    for (int idx = tid; idx < fam.nfinU * 4; idx += NT) finUL[idx] = fam.finU[idx];
    for (int idx = tid; idx < NRT * 2 * 16; idx += NT) slotL[idx] = slots[idx];
    // the tile's first barrier publishes the tables
    int bad = 0;
    if (!queue) {
        if (blockIdx.x < (unsigned)ntiles)
            quad_tile_any<NRT, NRTF, NKB, DLO, DHI>(fam, tiles[blockIdx.x], items, cu, cg, cpole, vx, store, hbuf, bad,
                                                    Xbuf, colmapL, dirsL, finUL, slotL);
    } else {
        for (;;) {
            if (tid == 0) next = atomicAdd(queue, 1);
            __syncthreads();
            const int ti = __builtin_amdgcn_readfirstlane(next);  // uniform: the tile's fields load into SGPRs
            __syncthreads();  // every thread has read `next` before it is overwritten
            if (ti >= ntiles) break;
            quad_tile_any<NRT, NRTF, NKB, DLO, DHI>(fam, tiles[ti], items, cu, cg, cpole, vx, store, hbuf, bad, Xbuf,
                                                    colmapL, dirsL, finUL, slotL);
        }
    }
    if (bad) atomicOr(err, bad);
}

template <int R, int RF, int KB, int DL, int DH>
hipError_t launch_quad_one(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                           const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                           uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int pgrid, int *queue,
                           hipStream_t stream) {
    constexpr size_t lds = QuadShape<R, KB, DH>::lds;
    hipError_t e = hipFuncSetAttribute((const void *)k_reduce_quad<R, RF, KB, DL, DH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int grid = ntiles;
    if (pgrid > 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = std::min(ntiles, std::max(1, cus) * pgrid);
    }
    hipLaunchKernelGGL((k_reduce_quad<R, RF, KB, DL, DH>), dim3(grid), dim3(64 * kQWaves), lds, stream, fam, items, tiles,
                       ntiles, pgrid > 0 ? queue : nullptr, cu, cg, cpole, vx, store, hbuf, slots, err);
    return hipGetLastError();
}

}  // namespace

// Shape of the quad kernel for a family: nrt row tiles (the first nrtf of
// them full quads), nkb K-blocks.  Quartic K3 surfaces: 11, 7, 7.
bool quad_shape(const DevFamily &fam, int &nrt, int &nrtf, int &nkb) {
    nkb = (fam.T + 31) / 32;
    nrt = 11;
    nrtf = 7;
    return fam.nv == 4 && fam.smask == 0xFu && fam.s == 220 && fam.T == 220 && fam.nsrc == 336 &&
           fam.ndir * fam.s <= kQTab && fam.ndir * 4 <= kQSmall && fam.nfinU * 4 <= kQSmall;
}

bool quad_supports_digits(int D) { return D == 7 || D == 9; }

// One launch for the tiles of every item, whatever its digit count (each
// item's DevDigitItem.D is 7 or 9; quad_supports_digits is checked on the host).
hipError_t launch_reduce_quad(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                              uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int pgrid, int *queue,
                              hipStream_t stream) {
    if (ntiles == 0) return hipSuccess;
    int nrt, nrtf, nkb;
    if (!quad_shape(fam, nrt, nrtf, nkb) || nkb != 7) return hipErrorInvalidValue;
    return launch_quad_one<11, 7, 7, 7, 9>(fam, items, tiles, ntiles, cu, cg, cpole, vx, store, hbuf, slots, err,
                                           pgrid, queue, stream);
}

}  // namespace crf
