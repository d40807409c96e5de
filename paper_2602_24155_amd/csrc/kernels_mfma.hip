// Exact int8-digit MFMA kernel for the controlled-reduction recurrence (gfx950).
//
// Same mathematics as k_reduce_chains (kernels.hip): each chain is one
// Frobenius start term reduced one pole order per step with
//   t  = psi[:, cols(v)] w                      (the decomposition of Proposition 3.3)
//   w' = sum_i (u_i + r_i + [i not in S]) t[src(r, i)]   (explicit R_{u,v}, Section 3.1)
// but t is computed for 32 chains at once as an integer matrix product on the
// matrix cores: the chain vectors are scattered into the target space of J_S
// (row v + g - 1_S), so chains with different directions share one product.
//
// Arithmetic: residues of Z/Q', Q' = B^D, B = p^e (B odd, B <= 169), held as
// D balanced base-B digits in int8.  psi (D digits, rows = J_S sources, cols =
// J_S targets) stays in VGPRs for the whole kernel; the 32 chain vectors are
// D int8 digit planes in LDS.  For each digit position k < D the products
// psi_i * X_j with i + j = k accumulate exactly in int32 (v_mfma_i32_32x32x32_i8);
// positions >= D are multiples of Q' and are skipped.  The D partial sums of
// each entry are recombined exactly in fp64 (Horner in two halves), reduced
// mod Q', gathered with the small integer weights, reduced again and split
// back into balanced digits for the next step.  Q' is a power of p that is a
// multiple of p^M, so the final values reduced mod p^M are the exact ones.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_layout.hpp"

namespace crf {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kCT = 32;  // chains per workgroup (one MFMA column tile)

__device__ __forceinline__ double mod_fp(double x, double Q, double invQ) {
    // exact for |x| < 2^53 and Q < 2^52: the fma result is the exact remainder
    double qt = floor(x * invQ);
    double r = fma(-qt, Q, x);
    if (r < 0) r += Q;
    if (r >= Q) r -= Q;
    return r;
}

// Algorithm 3 (greedy v) and the depth-first chunk length (largest k with
// U - k v >= 0, capped by the remaining pole orders).
__device__ static void choose_chunk2(const DevFamily &fam, const int *U, int poles_left, int *v, int &dir, int &k) {
    int left = fam.d;
    for (int i = 0; i < fam.nv; i++) v[i] = 0;
    for (int s = 0; s < fam.nv && left > 0; s++)
        if (((fam.smask >> s) & 1u) && U[s] != 0) {
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
        if (!moved) break;
    }
    k = poles_left;
    for (int i = 0; i < fam.nv; i++)
        if (v[i]) k = min(k, U[i] / v[i]);
    dir = -1;
    for (int t = 0; t < fam.ndir && dir < 0; t++) {
        bool eq = true;
        for (int i = 0; i < fam.nv; i++) eq = eq && (fam.dirs[t * fam.nv + i] == v[i]);
        if (eq) dir = t;
    }
}

constexpr int kTabCap = 2048;  // LDS capacity for colmap (ndir x s) entries
constexpr int kGCap = 512;     // LDS capacity for gsrc / gw (s x nv) entries

// Dynamic LDS layout (bytes):
//   X   : D digit planes x 32 chains x XS     int8  (chain vectors in the J_S target space)
//   Sb  : D positions x nsrc rows x 32 chains int32 (digit-position sums of t = psi x)
//   tables (colmap, gsrc, gw) and per-chain state
template <int NKB, int D>
__host__ __device__ constexpr size_t mfma_x_bytes() {
    return (size_t)D * kCT * (NKB * 32 + 16);
}

size_t mfma_lds_bytes_rt(int nkb, int D, int nsrc) {
    return (size_t)D * kCT * (nkb * 32 + 16) + (size_t)D * nsrc * kCT * 4 + kTabCap * 2 + 2 * kGCap * 2 +
           (size_t)kCT * 24 * 4;
}

template <int NRT, int NKB, int D>
__global__ __launch_bounds__(64 * NRT) void k_reduce_mfma(DevFamily fam, const DevDigitItem *__restrict__ items,
                                                          const DevTile *__restrict__ tiles,
                                                          const int16_t *__restrict__ cu,
                                                          const int32_t *__restrict__ cg,
                                                          const int32_t *__restrict__ cpole,
                                                          uint64_t *__restrict__ hbuf, int *__restrict__ err) {
    constexpr int K = NKB * 32;
    constexpr int XS = K + 16;  // bytes per (digit, chain) row of X
    constexpr int NT = 64 * NRT;
    constexpr int NGRP = NT / kCT;  // phase-3 row groups
    constexpr int DS = (D + 1) / 2;  // digit split: x = x_hi B^DS + x_lo
    extern __shared__ __align__(16) unsigned char lds[];
    const int s = fam.s, nv = fam.nv, nsrc = fam.nsrc, F = fam.F;
    const int n = fam.n;
    int8_t *X = reinterpret_cast<int8_t *>(lds);
    int *Sb = reinterpret_cast<int *>(lds + mfma_x_bytes<NKB, D>());
    int16_t *colmapL = reinterpret_cast<int16_t *>(Sb + (size_t)D * nsrc * kCT);
    int16_t *gsrcL = colmapL + kTabCap;
    int16_t *gwL = gsrcL + kGCap;
    int *U = reinterpret_cast<int *>(gwL + kGCap);
    int *V = U + kCT * 8;
    int *Dir = V + kCT * 8;
    int *Kleft = Dir + kCT;
    int *Pole = Kleft + kCT;
    int *Act = Pole + kCT;

    const DevTile tile = tiles[blockIdx.x];
    const DevDigitItem it = items[tile.item];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nch = tile.count;

    // psi digits of this wave's 32 source rows, resident for the whole kernel
    v4i A[D][NKB];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int kb = 0; kb < NKB; kb++)
            A[i][kb] = *reinterpret_cast<const v4i *>(it.apack + ((((size_t)wave * D + i) * NKB + kb) * 64 + lane) * 16);
    for (int idx = tid; idx < fam.ndir * s; idx += NT) colmapL[idx] = fam.colmap[idx];
    for (int idx = tid; idx < s * nv; idx += NT) {
        gsrcL[idx] = fam.gsrc[idx];
        gwL[idx] = fam.gw[idx];
    }
    for (int idx = tid; idx < (int)(mfma_x_bytes<NKB, D>() / 16); idx += NT)
        reinterpret_cast<v4i *>(X)[idx] = v4i{0, 0, 0, 0};
    for (int idx = tid; idx < nch * F; idx += NT) hbuf[(size_t)tile.chain0 * F + idx] = 0;
    __syncthreads();
    if (tid < nch) {
        const int g = tile.chain0 + tid;
        for (int i = 0; i < nv; i++) U[tid * 8 + i] = cu[(size_t)g * nv + i];
        Pole[tid] = cpole[g];
        int d0, k0;
        choose_chunk2(fam, &U[tid * 8], Pole[tid] - n, &V[tid * 8], d0, k0);
        if (d0 < 0 || k0 < 1) {
            atomicOr(err, 1);
            d0 = 0;
            Pole[tid] = n;
        }
        Dir[tid] = d0;
        Kleft[tid] = k0;
        const int col = colmapL[d0 * s + cg[g]];
        if (col < 0) atomicOr(err, 2);
        else X[tid * XS + col] = (int8_t)(1);  // balanced digits of 1: (1, 0, ..., 0)
    }
    __syncthreads();

    const double Bd = it.Bd, Qd = it.Qd, invQ = it.invQ, BHd = it.BHd, invBH = it.invBH, Bh = it.Bh;
    const double Bsplit = it.Bsplit, invBsplit = it.invBsplit, bias = it.bias;
    const int h = it.h, Bi = it.B, halfB = it.halfB, shift = it.shift;
    const uint32_t magic = it.magic;
    const bool z32 = it.z32 != 0;
    const int c3 = tid % kCT, g3 = tid / kCT;  // phase-3 chain and row group of this thread

    for (int step = 0; step < tile.steps; step++) {
        // ---- phase 1: digit products on the matrix cores; position sums to LDS
        {
            v16i acc[D];
#pragma unroll
            for (int k = 0; k < D; k++) acc[k] = v16i{0};
#pragma unroll
            for (int j = 0; j < D; j++) {
                v4i xb[NKB];
#pragma unroll
                for (int kb = 0; kb < NKB; kb++)
                    xb[kb] = *reinterpret_cast<const v4i *>(X + (j * kCT + (lane & 31)) * XS + kb * 32 + (lane >> 5) * 16);
#pragma unroll
                for (int i = 0; i + j < D; i++)
#pragma unroll
                    for (int kb = 0; kb < NKB; kb++)
                        acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i][kb], xb[kb], acc[i + j], 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int row = wave * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                if (row < nsrc)
#pragma unroll
                    for (int k = 0; k < D; k++) Sb[((size_t)k * nsrc + row) * kCT + (lane & 31)] = acc[k][r];
            }
        }
        __syncthreads();
        // ---- phase 2: chain bookkeeping; clear the digit planes
        if (tid < nch) {
            const int c = tid;
            Act[c] = Pole[c] > n;
            if (Act[c]) {
                for (int i = 0; i < nv; i++) U[c * 8 + i] -= V[c * 8 + i];
                Pole[c]--;
                Kleft[c]--;
                if (Pole[c] > n && Kleft[c] == 0) {
                    int d0, k0;
                    choose_chunk2(fam, &U[c * 8], Pole[c] - n, &V[c * 8], d0, k0);
                    if (d0 < 0 || k0 < 1) {
                        atomicOr(err, 1);
                        d0 = 0;
                        Pole[c] = n;
                    }
                    Dir[c] = d0;
                    Kleft[c] = k0;
                }
            }
        }
        for (int idx = tid; idx < (int)(mfma_x_bytes<NKB, D>() / 16); idx += NT)
            reinterpret_cast<v4i *>(X)[idx] = v4i{0, 0, 0, 0};
        __syncthreads();
        // ---- phase 3: Z_k[r] = sum_i (u_i + r_i + [i not in S]) S_k[src(r,i)]; w'[r] = sum_k Z_k B^k mod Q'
        if (c3 < nch && Act[c3]) {
            const int c = c3;
            const bool more = Pole[c] > n;
            const int16_t *cm = colmapL + Dir[c] * s;
            int Ucur[8];
            for (int i = 0; i < nv; i++) Ucur[i] = U[c * 8 + i];
            for (int r = g3; r < s; r += NGRP) {
                double z[D];
                if (z32) {
                    int zi[D];
#pragma unroll
                    for (int k = 0; k < D; k++) zi[k] = 0;
                    for (int i = 0; i < nv; i++) {
                        const int src = gsrcL[r * nv + i];
                        if (src < 0) continue;
                        const int wt = Ucur[i] + gwL[r * nv + i];
#pragma unroll
                        for (int k = 0; k < D; k++) zi[k] += wt * Sb[((size_t)k * nsrc + src) * kCT + c];
                    }
#pragma unroll
                    for (int k = 0; k < D; k++) z[k] = (double)zi[k];
                } else {
#pragma unroll
                    for (int k = 0; k < D; k++) z[k] = 0.0;
                    for (int i = 0; i < nv; i++) {
                        const int src = gsrcL[r * nv + i];
                        if (src < 0) continue;
                        const double wt = (double)(Ucur[i] + gwL[r * nv + i]);
#pragma unroll
                        for (int k = 0; k < D; k++) z[k] = fma(wt, (double)Sb[((size_t)k * nsrc + src) * kCT + c], z[k]);
                    }
                }
                double lo = 0.0, hi = 0.0;
#pragma unroll
                for (int k = D - 1; k >= 0; k--) {
                    if (k >= h) hi = fma(hi, Bd, z[k]);
                    else lo = fma(lo, Bd, z[k]);
                }
                double x = mod_fp(lo, Qd, invQ);
                x = fma(mod_fp(hi, BHd, invBH), Bh, x);
                if (x >= Qd) x -= Qd;
                if (x == 0.0) continue;
                if (more) {
                    const int col = cm[r];
                    if (col < 0) {
                        atomicOr(err, 2);
                        continue;
                    }
                    // balanced digits of x: unsigned digits of x + (Q'-1)/2, minus (B-1)/2
                    double xs = x + bias;
                    if (xs >= Qd) xs -= Qd;
                    double xh = floor(xs * invBsplit);
                    double rl = fma(-xh, Bsplit, xs);
                    if (rl < 0.0) {  // the rounded quotient was one too high
                        rl += Bsplit;
                        xh -= 1.0;
                    } else if (rl >= Bsplit) {
                        rl -= Bsplit;
                        xh += 1.0;
                    }
                    uint32_t vl = (uint32_t)rl, vh = (uint32_t)xh;
                    int8_t *xp = X + c * XS + col;
#pragma unroll
                    for (int j = 0; j < DS; j++) {
                        const uint32_t qd = __umulhi(vl, magic) >> shift;
                        xp[j * kCT * XS] = (int8_t)((int)(vl - qd * (uint32_t)Bi) - halfB);
                        vl = qd;
                    }
#pragma unroll
                    for (int j = DS; j < D; j++) {
                        const uint32_t qd = __umulhi(vh, magic) >> shift;
                        xp[j * kCT * XS] = (int8_t)((int)(vh - qd * (uint32_t)Bi) - halfB);
                        vh = qd;
                    }
                } else {
                    // pole n reached: numerator x^U g / x^S, reduced mod p^M
                    int Ui = -1;
                    for (int a = 0; a < fam.nfinU && Ui < 0; a++) {
                        bool eq = true;
                        for (int i = 0; i < nv; i++) eq = eq && (fam.finU[a * nv + i] == Ucur[i]);
                        if (eq) Ui = a;
                    }
                    const int f = Ui < 0 ? -1 : fam.finmap[Ui * s + r];
                    if (f < 0) atomicOr(err, 4);
                    else hbuf[(size_t)(tile.chain0 + c) * F + f] = (uint64_t)x % it.q;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_reduce_mfma4: same arithmetic as k_reduce_mfma, with the J_S source rows
// permuted (on the host) so that each output r of the weighted gather finds
// all its source rows in ONE lane's 16 accumulator rows.  The gather then
// runs on the MFMA accumulators directly: no LDS round trip for the digit
// sums.  Chain state lives in registers (every lane of a chain computes it
// identically) and the chain vectors are double buffered, so a step needs two
// barriers: after the products (the current vectors may be cleared) and after
// the new vectors are written.
// slots[bin*16 + j] (bin = 2*wave + lane/32) packs: bit0 valid, bit1 ends the
// output's group, bits 2-4 the variable i of the source row, bits 5-15 the
// constant weight r_i + [i not in S], bits 16-31 the output r.
template <int NV>
__device__ __forceinline__ static void choose_chunk_reg(const DevFamily &fam, const int8_t *dirsL, const int *U,
                                                        int poles_left, int *v, int &dir, int &k) {
    int left = fam.d;
#pragma unroll
    for (int i = 0; i < NV; i++) v[i] = 0;
#pragma unroll
    for (int sI = 0; sI < NV; sI++)
        if (left > 0 && ((fam.smask >> sI) & 1u) && U[sI] != 0) {
            v[sI] = 1;
            left--;
        }
    for (int guard = 0; guard < 64 && left > 0; guard++) {
        bool moved = false;
#pragma unroll
        for (int m = 0; m < NV; m++)
            if (left > 0 && v[m] < U[m]) {
                v[m]++;
                left--;
                moved = true;
            }
        if (!moved) break;
    }
    k = poles_left;
#pragma unroll
    for (int i = 0; i < NV; i++)
        if (v[i]) k = min(k, U[i] / v[i]);
    dir = -1;
    for (int t = 0; t < fam.ndir && dir < 0; t++) {
        bool eq = true;
#pragma unroll
        for (int i = 0; i < NV; i++) eq = eq && (dirsL[t * NV + i] == v[i]);
        if (eq) dir = t;
    }
}

// floor(u / v) for 0 <= u < 2^20 and 1 <= v <= 64: fp32 reciprocal estimate
// (off by at most one) and an exact integer correction
__device__ __forceinline__ static int div_small(int u, int v) {
    int q = (int)((float)u * __frcp_rn((float)v));
    q += (q + 1) * v <= u ? 1 : 0;
    q -= q * v > u ? 1 : 0;
    return q;
}

// Index of (v0, v1, deg - v0 - v1) among the monomials of degree deg in 3
// variables in lexicographically descending order, which is the family's
// order of directions (degree d) and of final exponents (degree |S| - 1): the
// monomials before it have a larger first exponent, (deg - v0)(deg - v0 + 1)/2
// of them, or the same first and a larger second one, deg - v0 - v1.
__device__ __forceinline__ static int mono_rank3(int v0, int v1, int deg) {
    const int r = deg - v0;
    return r * (r + 1) / 2 + (r - v1);
}

// choose_chunk_reg for 3 variables with the direction index in closed form
__device__ __forceinline__ static void choose_chunk3(const DevFamily &fam, const int *U, int poles_left, int *v,
                                                     int &dir, int &k) {
    int left = fam.d;
#pragma unroll
    for (int i = 0; i < 3; i++) v[i] = 0;
#pragma unroll
    for (int sI = 0; sI < 3; sI++)
        if (left > 0 && ((fam.smask >> sI) & 1u) && U[sI] != 0) {
            v[sI] = 1;
            left--;
        }
    for (int guard = 0; guard < 64 && left > 0; guard++) {
        bool moved = false;
#pragma unroll
        for (int m = 0; m < 3; m++)
            if (left > 0 && v[m] < U[m]) {
                v[m]++;
                left--;
                moved = true;
            }
        if (!moved) break;
    }
    k = poles_left;
#pragma unroll
    for (int i = 0; i < 3; i++)
        if (v[i]) k = min(k, div_small(U[i], v[i]));
    dir = left == 0 ? mono_rank3(v[0], v[1], fam.d) : -1;
}

// final-exponent index of U (3 variables, |U| = |S| - 1), -1 if U is not one
__device__ __forceinline__ static int fin_index3(const DevFamily &fam, const int *U) {
    const int deg = __popc(fam.smask & 7u) - 1;
    const bool ok = U[0] >= 0 && U[1] >= 0 && U[2] >= 0 && U[0] + U[1] + U[2] == deg;
    return ok ? mono_rank3(U[0], U[1], deg) : -1;
}

// Balanced base-B digits of x (0 <= x < Q') written to the D digit planes at xp
// (plane stride kCT * XS bytes).  x + bias is cut at B^DS so that both halves
// stay below 2^24 for the 32-bit magic division by B.
template <int D, int XS>
__device__ __forceinline__ static void put_digits(int8_t *xp, double x, double Qd, double bias, double Bsplit,
                                                  double invBsplit, uint32_t magic, int shift, int Bi, int halfB) {
    constexpr int DS = (D + 1) / 2;
    double xs = x + bias;
    if (xs >= Qd) xs -= Qd;
    double xh = floor(xs * invBsplit);
    double rl = fma(-xh, Bsplit, xs);
    if (rl < 0.0) {
        rl += Bsplit;
        xh -= 1.0;
    } else if (rl >= Bsplit) {
        rl -= Bsplit;
        xh += 1.0;
    }
    uint32_t vl = (uint32_t)rl, vh = (uint32_t)xh;
#pragma unroll
    for (int jd = 0; jd < DS; jd++) {
        const uint32_t qd = __umulhi(vl, magic) >> shift;
        xp[jd * kCT * XS] = (int8_t)((int)(vl - qd * (uint32_t)Bi) - halfB);
        vl = qd;
    }
#pragma unroll
    for (int jd = DS; jd < D; jd++) {
        const uint32_t qd = __umulhi(vh, magic) >> shift;
        xp[jd * kCT * XS] = (int8_t)((int)(vh - qd * (uint32_t)Bi) - halfB);
        vh = qd;
    }
}

// put_digits with the digit stride given at run time (one plane, or R2 bytes
// for a column of the folded last K-block)
template <int D>
__device__ __forceinline__ static void put_digits_st(int8_t *xp, int stride, double x, double Qd, double bias,
                                                     double Bsplit, double invBsplit, uint32_t magic, int shift,
                                                     int Bi, int halfB) {
    constexpr int DS = (D + 1) / 2;
    double xs = x + bias;
    if (xs >= Qd) xs -= Qd;
    double xh = floor(xs * invBsplit);
    double rl = fma(-xh, Bsplit, xs);
    if (rl < 0.0) {
        rl += Bsplit;
        xh -= 1.0;
    } else if (rl >= Bsplit) {
        rl -= Bsplit;
        xh += 1.0;
    }
    uint32_t vl = (uint32_t)rl, vh = (uint32_t)xh;
#pragma unroll
    for (int jd = 0; jd < DS; jd++) {
        const uint32_t qd = __umulhi(vl, magic) >> shift;
        xp[jd * stride] = (int8_t)((int)(vl - qd * (uint32_t)Bi) - halfB);
        vl = qd;
    }
#pragma unroll
    for (int jd = DS; jd < D; jd++) {
        const uint32_t qd = __umulhi(vh, magic) >> shift;
        xp[jd * stride] = (int8_t)((int)(vh - qd * (uint32_t)Bi) - halfB);
        vh = qd;
    }
}

// One tile (up to 32 vectors of one item) of the register-gather kernel.
// colmapL / dirsL hold the family tables and sl this lane's bin slots.
// One tile (up to 32 vectors of one item) of the register-gather kernel.
// colmapL / dirsL hold the family tables and sl this lane's bin slots.
template <int NRT, int NKB, int D, int NV, bool Z32>
__device__ __forceinline__ static void mfma4_tile(const DevFamily &fam, const DevTile &tile,
                                                  const DevDigitItem *__restrict__ items,
                                                  const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
                                                  const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx,
                                                  uint64_t *__restrict__ store, uint64_t *__restrict__ hbuf,
                                                  const uint32_t (&sl)[16], int *__restrict__ err, int8_t *Xbuf,
                                                  const int16_t *colmapL, const int8_t *dirsL) {
    constexpr int K = NKB * 32;
    constexpr int XS = K + 16;
    constexpr int NT = 64 * NRT;
    constexpr int XB = D * kCT * XS;  // bytes of one set of digit planes
    const int s = fam.s, F = fam.F, n = fam.n;
    const DevDigitItem it = items[tile.item];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 31, half = lane >> 5, bin = 2 * wave + half;
    const int nch = tile.count;

    v4i A[D][NKB];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int kb = 0; kb < NKB; kb++)
            A[i][kb] = *reinterpret_cast<const v4i *>(it.apack + ((((size_t)wave * D + i) * NKB + kb) * 64 + lane) * 16);
    for (int idx = tid; idx < 2 * XB / 16; idx += NT) reinterpret_cast<v4i *>(Xbuf)[idx] = v4i{0, 0, 0, 0};
    for (int idx = tid; idx < nch * F; idx += NT)
        if (vx[tile.chain0 + idx / F].out < 0) hbuf[(size_t)tile.chain0 * F + idx] = 0;
    for (int idx = tid; idx < nch * s; idx += NT) {
        const int out = vx[tile.chain0 + idx / s].out;
        if (out >= 0) store[(size_t)out * s + idx % s] = 0;
    }
    __syncthreads();

    const double Bd = it.Bd, Qd = it.Qd, invQ = it.invQ, BHd = it.BHd, invBH = it.invBH, Bh = it.Bh;
    const double Bsplit = it.Bsplit, invBsplit = it.invBsplit, bias = it.bias;
    const int Bi = it.B, halfB = it.halfB, shift = it.shift;
    const uint32_t magic = it.magic;
    const double qd = (double)it.q, invq = 1.0 / qd;  // p^M < Q' < 2^52: mod_fp is exact

    // chain state (registers; identical in every lane of chain c)
    int U[NV], V[NV], dir = 0, kleft = 0, pole = n, pend = n, vout = -1;
#pragma unroll
    for (int i = 0; i < NV; i++) U[i] = V[i] = 0;
    if (c < nch) {
        const int g = tile.chain0 + c;
        const DevVec xv = vx[g];
#pragma unroll
        for (int i = 0; i < NV; i++) U[i] = cu[(size_t)g * NV + i];
        pole = cpole[g];
        pend = xv.pend;
        vout = xv.out;
        int d0, k0;
        if (xv.dir >= 0) {  // one forced direction for the whole range
            d0 = xv.dir;
            k0 = pole - pend;
#pragma unroll
            for (int i = 0; i < NV; i++) V[i] = dirsL[d0 * NV + i];
        } else {
            choose_chunk_reg<NV>(fam, dirsL, U, pole - pend, V, d0, k0);
        }
        if (d0 < 0 || k0 < 1) {
            if (wave == 0 && half == 0) atomicOr(err, 1);
            d0 = 0;
            pole = pend;
        }
        dir = d0;
        kleft = k0;
        if (xv.in < 0) {
            if (wave == 0 && half == 0) {
                const int col = colmapL[d0 * s + cg[g]];
                if (col < 0) atomicOr(err, 2);
                else Xbuf[c * XS + col] = (int8_t)1;  // balanced digits of 1
            }
        } else {
            // start vector from the store: the lanes of chain c split its entries
            for (int r = bin; r < s; r += 2 * NRT) {
                const uint64_t x = store[(size_t)xv.in * s + r];
                if (x == 0) continue;
                const int col = colmapL[d0 * s + r];
                if (col < 0) {
                    atomicOr(err, 2);
                    continue;
                }
                put_digits<D, XS>(Xbuf + c * XS + col, (double)x, Qd, bias, Bsplit, invBsplit, magic, shift, Bi,
                                  halfB);
            }
        }
    }
    __syncthreads();
    int cur = 0;

    for (int step = 0; step < tile.steps; step++) {
        const int8_t *Xc = Xbuf + cur * XB;
        int8_t *Xn = Xbuf + (cur ^ 1) * XB;
        v16i acc[D];
#pragma unroll
        for (int k = 0; k < D; k++) acc[k] = v16i{0};
#pragma unroll
        for (int j = 0; j < D; j++) {
            v4i xb[NKB];
#pragma unroll
            for (int kb = 0; kb < NKB; kb++)
                xb[kb] = *reinterpret_cast<const v4i *>(Xc + (j * kCT + c) * XS + kb * 32 + half * 16);
#pragma unroll
            for (int i = 0; i + j < D; i++)
#pragma unroll
                for (int kb = 0; kb < NKB; kb++)
                    acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i][kb], xb[kb], acc[i + j], 0, 0, 0);
        }
        // bookkeeping of this lane's chain: exponent after the step, next direction
        const bool act = pole > pend;
        int up[NV], Vn[NV], dirn = dir, kleftn = kleft - 1;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            up[i] = U[i] - (act ? V[i] : 0);
            Vn[i] = V[i];
        }
        const bool more = act && pole - 1 > pend;
        if (more && kleftn == 0) {
            int d0, k0;
            choose_chunk_reg<NV>(fam, dirsL, up, pole - 1 - pend, Vn, d0, k0);
            if (d0 < 0 || k0 < 1) {
                atomicOr(err, 1);
                d0 = 0;
                k0 = 1 << 30;
            }
            dirn = d0;
            kleftn = k0;
        }
        // a chain that ends here at pole n: row of its final exponent in finmap
        int fin_row = -1;
        if (act && !more && vout < 0) {
            int Ui = -1;
            for (int a = 0; a < fam.nfinU && Ui < 0; a++) {
                bool eq = true;
#pragma unroll
                for (int i = 0; i < NV; i++) eq = eq && (fam.finU[a * NV + i] == up[i]);
                if (eq) Ui = a;
            }
            if (Ui < 0) atomicOr(err, 4);
            else fin_row = Ui * s;
        }
        __syncthreads();  // every wave has read the current digit planes
        if (act) {
            const int16_t *cm = colmapL + dirn * s;
            // the lane's slots in groups of the constant pattern: accumulate the
            // weighted digit sums of a group, then finish its output r
            int j0 = 0;
#pragma unroll
            for (int g = 0; g < slot_groups(NRT); g++) {
                const int gs = slot_group(NRT, g);
                int zi[D];
                double zd[D];
#pragma unroll
                for (int k = 0; k < D; k++) {
                    zi[k] = 0;
                    zd[k] = 0.0;
                }
                uint32_t wend = 0;
#pragma unroll
                for (int m = 0; m < 3; m++) {
                    if (m >= gs) break;
                    const int j = j0 + m;
                    const uint32_t w = sl[j];
                    wend = w;
                    // variable of the slot: m in a three-row group, the reserved z in a one-row group
                    const int iv = slot_var(NRT, g) < 0 ? m : slot_var(NRT, g);
                    const int wt = up[iv] + (int)((w >> 5) & 2047u);  // empty slots meet zero rows
                    if (Z32) {
#pragma unroll
                        for (int k = 0; k < D; k++) zi[k] += __mul24(wt, acc[k][j]);
                    } else {
#pragma unroll
                        for (int k = 0; k < D; k++) zd[k] = fma((double)wt, (double)acc[k][j], zd[k]);
                    }
                }
                j0 += gs;
                // output r complete: w'[r] = sum_k Z_k B^k mod Q'
                const int r = (int)(wend >> 16);
                constexpr int H = D / 2;  // Horner split (host checks both halves stay exact)
                double lo = 0.0, hi = 0.0;
#pragma unroll
                for (int k = D - 1; k >= 0; k--) {
                    const double zk = Z32 ? (double)zi[k] : zd[k];
                    if (k >= H) hi = fma(hi, Bd, zk);
                    else lo = fma(lo, Bd, zk);
                }
                double x = mod_fp(lo, Qd, invQ);
                x = fma(mod_fp(hi, BHd, invBH), Bh, x);
                if (x >= Qd) x -= Qd;
                if (r == 0xFFFF) continue;  // unused group slot
                if (more) {
                    const int col = cm[r];
                    if (col < 0) {
                        if (x != 0.0) atomicOr(err, 2);
                        continue;
                    }
                    put_digits<D, XS>(Xn + c * XS + col, x, Qd, bias, Bsplit, invBsplit, magic, shift, Bi, halfB);
                } else if (x != 0.0) {
                    if (vout >= 0) {
                        store[(size_t)vout * s + r] = (uint64_t)mod_fp(x, qd, invq);  // combine point
                    } else if (fin_row >= 0) {
                        const int f = fam.finmap[fin_row + r];
                        if (f < 0) atomicOr(err, 4);
                        else hbuf[(size_t)(tile.chain0 + c) * F + f] = (uint64_t)mod_fp(x, qd, invq);
                    }
                }
            }
        }
        // clear the planes just consumed; they receive the vectors of the next step
        int8_t *Xz = Xbuf + cur * XB;
        for (int idx = tid; idx < XB / 16; idx += NT) reinterpret_cast<v4i *>(Xz)[idx] = v4i{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < NV; i++) {
            U[i] = up[i];
            V[i] = Vn[i];
        }
        if (act) {
            pole -= 1;
            dir = dirn;
            kleft = kleftn;
        }
        cur ^= 1;
        __syncthreads();  // next digit planes complete
    }
}

template <int NRT, int NKB, int D, int NV, bool Z32>
__device__ __forceinline__ static void mfma4_prologue(const DevFamily &fam, const uint32_t *__restrict__ slots,
                                                      uint32_t (&sl)[16], int16_t *colmapL, int8_t *dirsL) {
    constexpr int NT = 64 * NRT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, bin = 2 * wave + (lane >> 5);
#pragma unroll
    for (int j = 0; j < 16; j++) sl[j] = slots[bin * 16 + j];
    for (int idx = tid; idx < fam.ndir * fam.s; idx += NT) colmapL[idx] = fam.colmap[idx];
    for (int idx = tid; idx < fam.ndir * fam.nv; idx += NT) dirsL[idx] = fam.dirs[idx];
    // the tile body's first barrier publishes the tables
}

// One workgroup per tile.
template <int NRT, int NKB, int D, int NV, bool Z32>
__global__ __launch_bounds__(64 * NRT) void k_reduce_mfma4(DevFamily fam, const DevDigitItem *__restrict__ items,
                                                           const DevTile *__restrict__ tiles,
                                                           const int16_t *__restrict__ cu,
                                                           const int32_t *__restrict__ cg,
                                                           const int32_t *__restrict__ cpole,
                                                           const DevVec *__restrict__ vx,
                                                           uint64_t *__restrict__ store,
                                                           uint64_t *__restrict__ hbuf,
                                                           const uint32_t *__restrict__ slots, int *__restrict__ err) {
    constexpr int XB = D * kCT * (NKB * 32 + 16);
    __shared__ __align__(16) int8_t Xbuf[2 * XB];
    __shared__ int16_t colmapL[kTabCap];
    __shared__ int8_t dirsL[512];
    uint32_t sl[16];
    mfma4_prologue<NRT, NKB, D, NV, Z32>(fam, slots, sl, colmapL, dirsL);
    mfma4_tile<NRT, NKB, D, NV, Z32>(fam, tiles[blockIdx.x], items, cu, cg, cpole, vx, store, hbuf, sl, err, Xbuf,
                                     colmapL, dirsL);
}

// Persistent form: a grid sized to the resident capacity of the device drains
// the tile list through an atomic counter (*queue, zero at launch).  Tiles
// are ordered longest first, so the last tiles taken are the short ones.
// Every workgroup leaves the loop once the counter passes ntiles.
template <int NRT, int NKB, int D, int NV, bool Z32>
__global__ __launch_bounds__(64 * NRT) void k_reduce_mfma4_persistent(
    DevFamily fam, const DevDigitItem *__restrict__ items, const DevTile *__restrict__ tiles, int ntiles,
    int *__restrict__ queue, const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
    const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx, uint64_t *__restrict__ store,
    uint64_t *__restrict__ hbuf, const uint32_t *__restrict__ slots, int *__restrict__ err) {
    constexpr int XB = D * kCT * (NKB * 32 + 16);
    __shared__ __align__(16) int8_t Xbuf[2 * XB];
    __shared__ int16_t colmapL[kTabCap];
    __shared__ int8_t dirsL[512];
    __shared__ int next;
    uint32_t sl[16];
    mfma4_prologue<NRT, NKB, D, NV, Z32>(fam, slots, sl, colmapL, dirsL);
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        const int ti = next;
        __syncthreads();  // every thread has read `next` before it is overwritten
        if (ti >= ntiles) break;
        mfma4_tile<NRT, NKB, D, NV, Z32>(fam, tiles[ti], items, cu, cg, cpole, vx, store, hbuf, sl, err, Xbuf,
                                         colmapL, dirsL);
    }
}

__global__ void k_zero_ints(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_reduce_mfma5: the register-gather kernel with two tiles of one
// hypersurface per workgroup, interleaved so that the matrix cores and the
// vector ALUs work at the same time.  A step alternates two phases, each a
// straight-line block closed by one barrier:
//   phase 1: products of tile B (step t)   || finish of tile A (step t)
//   phase 2: products of tile A (step t+1) || finish of tile B (step t)
// The finish of a tile (weighted gather, digit split) is branch-free: the new
// digits come from a carry propagation over the digit-position sums (no
// recombination), a digit that has nowhere to go is
// written to the pad column of its plane row (never read by the products),
// and the digits of a chain that ends at this step are parked at column r of
// its own rows of the next planes (which no later step of that chain reads),
// then turned into residues and written out after the barrier.
template <int NV>
struct TileState {
    int U[NV], V[NV];
    int dir, kleft, pole, pend, vout, fin_row;
    bool act, more;
    int up[NV], Vn[NV], dirn, kleftn;
};

template <int NRT, int NKB, int D, int NV>
__device__ static void mfma5_init(const DevFamily &fam, const DevTile &tile, const DevDigitItem &it,
                                  const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
                                  const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx,
                                  uint64_t *__restrict__ store, int *__restrict__ err, int8_t *X,
                                  const int16_t *colmapL, const int8_t *dirsL, TileState<NV> &ts) {
    static_assert(NV == 3, "the direction index is in closed form for 3 variables");
    constexpr int XS = NKB * 32 + 16;
    const int s = fam.s, n = fam.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 31, half = lane >> 5, bin = 2 * wave + half;
#pragma unroll
    for (int i = 0; i < NV; i++) ts.U[i] = ts.V[i] = 0;
    ts.dir = 0;
    ts.kleft = 0;
    ts.pole = n;
    ts.pend = n;
    ts.vout = -1;
    if (c >= tile.count) return;
    const int g = tile.chain0 + c;
    const DevVec xv = vx[g];
#pragma unroll
    for (int i = 0; i < NV; i++) ts.U[i] = cu[(size_t)g * NV + i];
    ts.pole = cpole[g];
    ts.pend = xv.pend;
    ts.vout = xv.out;
    int d0, k0;
    if (xv.dir >= 0) {
        d0 = xv.dir;
        k0 = ts.pole - ts.pend;
#pragma unroll
        for (int i = 0; i < NV; i++) ts.V[i] = dirsL[d0 * NV + i];
    } else {
        choose_chunk3(fam, ts.U, ts.pole - ts.pend, ts.V, d0, k0);
    }
    if (d0 < 0 || k0 < 1) {
        if (wave == 0 && half == 0) atomicOr(err, 1);
        d0 = 0;
        ts.pole = ts.pend;
    }
    ts.dir = d0;
    ts.kleft = k0;
    const double Qd = it.Qd, bias = it.bias, Bsplit = it.Bsplit, invBsplit = it.invBsplit;
    if (xv.in < 0) {
        if (wave == 0 && half == 0) {
            const int col = colmapL[d0 * s + cg[g]];
            if (col < 0) atomicOr(err, 2);
            else X[c * XS + col] = (int8_t)1;  // balanced digits of 1
        }
    } else {
        for (int r = bin; r < s; r += 2 * NRT) {
            const uint64_t x = store[(size_t)xv.in * s + r];
            if (x == 0) continue;
            const int col = colmapL[d0 * s + r];
            if (col < 0) {
                atomicOr(err, 2);
                continue;
            }
            const int stride = col >= 32 * (NKB - 1) ? fam.T - 32 * (NKB - 1) : kCT * XS;  // folded last block
            put_digits_st<D>(X + c * XS + col, stride, (double)x, Qd, bias, Bsplit, invBsplit, it.magic, it.shift,
                             it.B, it.halfB);
        }
    }
}

// exponent after the step, next direction and chunk, final-exponent row
template <int NV>
__device__ __forceinline__ static void mfma5_book(const DevFamily &fam, TileState<NV> &ts, int &bad) {
    ts.act = ts.pole > ts.pend;
    ts.dirn = ts.dir;
    ts.kleftn = ts.kleft - 1;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        ts.up[i] = ts.U[i] - (ts.act ? ts.V[i] : 0);
        ts.Vn[i] = ts.V[i];
    }
    ts.more = ts.act && ts.pole - 1 > ts.pend;
    if (ts.more && ts.kleftn == 0) {
        int d0, k0;
        choose_chunk3(fam, ts.up, ts.pole - 1 - ts.pend, ts.Vn, d0, k0);
        if (d0 < 0 || k0 < 1) {
            bad |= 1;
            d0 = 0;
            k0 = 1 << 30;
        }
        ts.dirn = d0;
        ts.kleftn = k0;
    }
    ts.fin_row = -1;
    if (ts.act && !ts.more && ts.vout < 0) {
        const int Ui = fin_index3(fam, ts.up);
        if (Ui < 0) bad |= 4;
        else ts.fin_row = Ui * fam.s;
    }
}

template <int NV>
__device__ __forceinline__ static void mfma5_advance(TileState<NV> &ts) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
        ts.U[i] = ts.up[i];
        ts.V[i] = ts.Vn[i];
    }
    if (ts.act) {
        ts.pole -= 1;
        ts.dir = ts.dirn;
        ts.kleft = ts.kleftn;
    }
}

// One accumulator element of the finished tile, read straight from its
// accumulation register (AGPR): this keeps the finished accumulator in AGPRs
// while the other tile's MFMAs fill other AGPRs, instead of the whole
// accumulator being copied to VGPRs before each phase.  Each element is read
// at least one barrier after the MFMA that wrote it.
__device__ __forceinline__ static int agpr_read(int x) {
    int v;
    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(v) : "a"(x));
    return v;
}

template <int NKB, int D>
__device__ __forceinline__ static void mfma5_products(const v4i (&A)[D][NKB], const int8_t *Xc, int c, int half,
                                                      v16i (&acc)[D]) {
    constexpr int XS = NKB * 32 + 16;
#pragma unroll
    for (int k = 0; k < D; k++) acc[k] = v16i{0};
#pragma unroll
    for (int j = 0; j < D; j++) {
        v4i xb[NKB];
#pragma unroll
        for (int kb = 0; kb < NKB; kb++)
            xb[kb] = *reinterpret_cast<const v4i *>(Xc + (j * kCT + c) * XS + kb * 32 + half * 16);
#pragma unroll
        for (int i = 0; i + j < D; i++)
#pragma unroll
            for (int kb = 0; kb < (j == 0 ? NKB : NKB - 1); kb++)  // the last block is folded into plane 0
                acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i][kb], xb[kb], acc[i + j], 0, 0, 0);
    }
}

// The finish of one output group of a tile's step is split into 1 + 2D
// pieces: an init piece (slot weights, destination), then per digit position
// k a gather piece (z_k = sum over the group's slots of weight * product sum)
// and a carry piece.  Digits of continuing chains go to their columns of the
// next planes, those of a chain that ends at this step are parked at column r
// of its own rows there, everything else goes to the pad column K.  The state
// between the pieces of a group is a FinState.
struct FinState {
    int wt[3];
    int zi;          // z_k (32-bit sums)
    double zd;       // z_k (wider sums)
    double carry;    // carry into position k (wider sums)
    int ci;          // carry into position k (32-bit sums)
    int nz;          // OR of the digits: the balanced digits of 0 mod Q' are all 0
    int8_t *dst;     // where the next digit goes
    int stride;      // to the next digit: one plane, or R2 bytes for a folded column
    int r2;          // target rows in the folded last K-block
    bool chk;        // continuing chain whose output has no column under its direction
};

constexpr int slot_first(int nrt, int g) {  // first slot of output group g
    int t = 0;
    for (int q = 0; q < g; q++) t += slot_group(nrt, q);
    return t;
}

template <int D>
constexpr int pieces_per_group() { return 1 + 2 * D; }

template <int NRT, int NKB, int D, int NV, bool Z32, int P>
__device__ __forceinline__ static void mfma5_piece(const v16i (&acc)[D], const uint32_t (&sl)[16],
                                                   const TileState<NV> &ts, const int (&cols)[9], int8_t *row,
                                                   const DevDigitItem &it, FinState &fs, int &bad) {
    constexpr int K = NKB * 32;
    constexpr int XS = K + 16;
    constexpr int G = P / pieces_per_group<D>(), w = P % pieces_per_group<D>();
    constexpr int gs = slot_group(NRT, G);
    constexpr int j0 = slot_first(NRT, G);
    if constexpr (w == 0) {  // init
        const bool cont = ts.act && ts.more, ends = ts.act && !ts.more;
#pragma unroll
        for (int m = 0; m < gs; m++) {
            const int iv = slot_var(NRT, G) < 0 ? m : slot_var(NRT, G);
            fs.wt[m] = ts.up[iv] + (int)((sl[j0 + m] >> 5) & 2047u);
        }
        const int r = (int)(sl[j0 + gs - 1] >> 16);
        const bool rv = r != 0xFFFF;
        const int col = cols[G];
        const bool put = cont && rv && col >= 0;
        const bool park = ends && rv;
        fs.dst = row + (put ? col : (park ? r : K));
        fs.stride = (put && col >= 32 * (NKB - 1)) ? fs.r2 : kCT * XS;
        fs.carry = 0.0;
        fs.ci = 0;
        fs.nz = 0;
        fs.chk = cont && rv && col < 0;
    } else if constexpr (w % 2 == 1) {  // gather of position k
        constexpr int k = (w - 1) / 2;
        if constexpr (Z32) {
            int z = 0;
#pragma unroll
            for (int m = 0; m < gs; m++) z += __mul24(fs.wt[m], agpr_read(acc[k][j0 + m]));
            fs.zi = z;
        } else {
            double z = 0.0;
#pragma unroll
            for (int m = 0; m < gs; m++) z = fma((double)fs.wt[m], (double)agpr_read(acc[k][j0 + m]), z);
            fs.zd = z;
        }
    } else {  // carry step at position k
        constexpr int k = (w - 2) / 2;
        // t = z_k + carry, carry = round(t / B), d_k = t - B carry (|d_k| <=
        // (B-1)/2 since B is odd); the carry out of position D - 1 is a
        // multiple of Q' and is dropped.  round() adds 1.5 2^52: the sum then
        // lies in [2^52, 2^53), where the unit in the last place is 1, so its
        // mantissa is 2^51 + round(t / B).  For |t| < 2^31 (Z32: the host
        // bounds the carry sums too) the error of the product (< 2^-23) cannot
        // carry t / B across a half-integer (t / B lies at least 1 / (2B) from
        // one), so the rounding is exact; the carry is then the low word of
        // the sum (two's complement, as 2^51 is 0 mod 2^32), and the digit is
        // only needed mod 2^8 (|d_k| < 128), where a 24-bit multiply-add gives
        // it.  For wider sums the carry stays in fp64 and a range test fixes
        // the one-unit error the rounding can make.
        const double Bd = it.Bd, invB = 1.0 / Bd;
        constexpr double kRound = 6755399441055744.0;  // 1.5 2^52
        if constexpr (Z32) {
            const int t = fs.zi + fs.ci;
            fs.ci = __double2loint(fma((double)t, invB, kRound));
            // low 24 bits of the carry times 2^24 - B, plus t: = d_k mod 2^8.
            // Written out because, with only 8 result bits in use, the
            // compiler would otherwise narrow it to a quarter-rate 32-bit mul.
            unsigned du;
            asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(du) : "v"(fs.ci), "v"((1u << 24) - (unsigned)it.B), "v"(t));
            fs.nz |= (int)(du & 0xffu);
            *fs.dst = (int8_t)du;
        } else {
            const double t = fs.zd + fs.carry;
            double q = fma(t, invB, kRound) - kRound;
            double dk = fma(-q, Bd, t);
            const double hB = (double)it.halfB;
            const double up1 = (double)(dk > hB), dn1 = (double)(dk < -hB);
            q += up1 - dn1;
            dk += Bd * (dn1 - up1);
            fs.carry = q;
            const int di = (int)dk;
            fs.nz |= di;
            *fs.dst = (int8_t)di;
        }
        fs.dst += fs.stride;
        if constexpr (k == D - 1) bad |= (fs.chk && fs.nz != 0) ? 2 : 0;
    }
}

template <int NRT, int NKB, int D, int NV, bool Z32, int P, int P1>
__device__ __forceinline__ static void mfma5_pieces(const v16i (&acc)[D], const uint32_t (&sl)[16],
                                                    const TileState<NV> &ts, const int (&cols)[9], int8_t *row,
                                                    const DevDigitItem &it, FinState &fs, int &bad) {
    if constexpr (P < P1) {
        mfma5_piece<NRT, NKB, D, NV, Z32, P>(acc, sl, ts, cols, row, it, fs, bad);
        mfma5_pieces<NRT, NKB, D, NV, Z32, P + 1, P1>(acc, sl, ts, cols, row, it, fs, bad);
    }
}

// The products of a phase as a list of units, one MFMA each: plane J
// (products with digit J of the chains' vectors) holds the units (kb, i),
// kb major, so consecutive MFMAs feed different accumulators.
//
// The last K-block holds only the R2 = T - 32 (NKB - 1) target rows past the
// full blocks: they are stored folded, digit J of row 32 (NKB - 1) + t at
// byte 32 (NKB - 1) + R2 J + t of plane 0's row (R2 D <= 32), and the psi
// fragments of that block are A'_m[:, R2 J + t] = digit m - J of psi[:, 32
// (NKB - 1) + t] (J <= m).  One product A'_m x (plane 0's last block) then
// gives the whole last-block contribution to accumulator m, so planes J >= 1
// have no last-block units.
template <int D, int NKB>
struct UnitMap {
    static constexpr int blocks(int J) { return J == 0 ? NKB : NKB - 1; }
    static constexpr int count = D * NKB + D * (D - 1) / 2 * (NKB - 1);
    static constexpr int plane(int u) {
        int J = 0;
        while (u >= (D - J) * blocks(J)) u -= (D - J) * blocks(J), J++;
        return J;
    }
    static constexpr int first(int J) {  // first unit of plane J
        int t = 0;
        for (int q = 0; q < J; q++) t += (D - q) * blocks(q);
        return t;
    }
    // The operands of plane J (J >= 1) are read from LDS kLead units before
    // the plane starts (never before plane J - 1 starts: the buffer they go to
    // is plane J - 2's): far enough ahead to hide the LDS latency, close
    // enough that few digit stores of the finishing work are issued in between
    // (the LDS counter tracks at most 15 outstanding operations).
    static constexpr int kLead = 4;
    static constexpr int load_unit(int J) {
        const int u = first(J) - kLead;
        return u > first(J - 1) ? u : first(J - 1);
    }
    static constexpr int plane_loaded_at(int u) {  // plane whose operands unit u reads, or -1
        for (int J = 1; J < D; J++)
            if (load_unit(J) == u) return J;
        return -1;
    }
};

// One unit of a phase: the MFMA of tile P's unit U, the finishing pieces of
// tile F and the plane clearing stores that fall on it, then a scheduling
// fence, so that each MFMA runs in the shadow of independent vector work.
template <int NRT, int NKB, int D, int NV, bool Z32, int U>
__device__ __forceinline__ static void mfma5_unit(const v4i (&A)[D][NKB], const int8_t *Xp, int c, int half,
                                                  v4i (&xb)[2][NKB], v16i (&accP)[D], const v16i (&accF)[D],
                                                  const uint32_t (&sl)[16], const TileState<NV> &tsF,
                                                  const int (&cols)[9], int8_t *rowF, const DevDigitItem &it,
                                                  FinState &fs, v4i *Xz, int tid, int &bad) {
    using UM = UnitMap<D, NKB>;
    constexpr int NU = UM::count;
    if constexpr (U < NU) {
        constexpr int XS = NKB * 32 + 16;
        constexpr int J = UM::plane(U);
        constexpr int w = U - UM::first(J);
        constexpr int kb = w / (D - J), i = w % (D - J);
        constexpr int JL = UM::plane_loaded_at(U);
        if constexpr (JL > 0) {
#pragma unroll
            for (int b = 0; b < NKB - 1; b++)
                xb[JL & 1][b] = *reinterpret_cast<const v4i *>(Xp + (JL * kCT + c) * XS + b * 32 + half * 16);
        }
        accP[i + J] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i][kb], xb[J & 1][kb], accP[i + J], 0, 0, 0);
        constexpr int NP = slot_groups(NRT) * pieces_per_group<D>();
        mfma5_pieces<NRT, NKB, D, NV, Z32, U * NP / NU, (U + 1) * NP / NU>(accF, sl, tsF, cols, rowF, it, fs, bad);
        // plane clearing: NZ 16-byte stores per thread, spread over the phase
        constexpr int NT = 64 * NRT;
        constexpr int N16 = D * kCT * XS / 16;
        constexpr int NZ = (N16 + NT - 1) / NT;
        static_assert(NU >= NZ, "clearing stores per phase");
        if constexpr (U % (NU / NZ) == 0 && U / (NU / NZ) < NZ) {
            constexpr int zq = U / (NU / NZ);
            if constexpr (N16 % NT == 0) Xz[zq * NT + tid] = v4i{0, 0, 0, 0};
            else if (zq * NT + tid < N16) Xz[zq * NT + tid] = v4i{0, 0, 0, 0};
        }
        __builtin_amdgcn_sched_barrier(0);
        mfma5_unit<NRT, NKB, D, NV, Z32, U + 1>(A, Xp, c, half, xb, accP, accF, sl, tsF, cols, rowF, it, fs, Xz, tid,
                                                bad);
    }
}

// One phase: the products of tile P (planes Xp -> accP) interleaved with the
// finish of tile F (accF -> planes rowF) and the clearing of the planes Xz.
template <int NRT, int NKB, int D, int NV, bool Z32>
__device__ __forceinline__ static void mfma5_phase(const v4i (&A)[D][NKB], const int8_t *Xp, int c, int half,
                                                   v16i (&accP)[D], const v16i (&accF)[D], const uint32_t (&sl)[16],
                                                   const TileState<NV> &tsF, const int16_t *cm, int8_t *rowF,
                                                   const DevDigitItem &it, int8_t *Xz, int tid, int r2, int &bad) {
    constexpr int XS = NKB * 32 + 16;
    constexpr int G = slot_groups(NRT);
    static_assert(G <= 9, "slot groups");
    int cols[9];
#pragma unroll
    for (int g = 0; g < G; g++) {
        const int r = (int)(sl[slot_first(NRT, g) + slot_group(NRT, g) - 1] >> 16);
        cols[g] = cm[r != 0xFFFF ? r : 0];
    }
    v4i xb[2][NKB];
#pragma unroll
    for (int b = 0; b < NKB; b++) xb[0][b] = *reinterpret_cast<const v4i *>(Xp + c * XS + b * 32 + half * 16);
#pragma unroll
    for (int k = 0; k < D; k++) accP[k] = v16i{0};
    FinState fs;
    fs.r2 = r2;
    mfma5_unit<NRT, NKB, D, NV, Z32, 0>(A, Xp, c, half, xb, accP, accF, sl, tsF, cols, rowF, it, fs,
                                        reinterpret_cast<v4i *>(Xz), tid, bad);
}

// After the barrier: the parked outputs of the chains that ended go out.
template <int NRT, int NKB, int D, int NV>
__device__ __forceinline__ static void mfma5_flush(const DevFamily &fam, const TileState<NV> &ts, const int8_t *Xn,
                                                   int c, int bin, int chain0, const DevDigitItem &it,
                                                   uint64_t *__restrict__ store, uint64_t *__restrict__ hbuf,
                                                   int &bad) {
    constexpr int XS = NKB * 32 + 16;
    if (!(ts.act && !ts.more)) return;
    const int s = fam.s;
    const double qd = (double)it.q, invq = 1.0 / qd, Bd = it.Bd, Qd = it.Qd;
    for (int r = bin; r < s; r += 2 * NRT) {
        // x = sum_k d_k B^k from the digits parked at column r (|x| < Q' / 2)
        double x = 0.0;
        for (int k = D - 1; k >= 0; k--) x = fma(x, Bd, (double)Xn[k * kCT * XS + c * XS + r]);
        if (x < 0.0) x += Qd;
        if (x == 0.0) continue;
        const uint64_t v = (uint64_t)mod_fp(x, qd, invq);
        if (ts.vout >= 0) {
            store[(size_t)ts.vout * s + r] = v;
        } else if (ts.fin_row >= 0) {
            const int f = fam.finmap[ts.fin_row + r];
            if (f < 0) bad |= 4;
            else hbuf[(size_t)(chain0 + c) * fam.F + f] = v;
        }
    }
}

template <int NRT, int NKB, int D>
constexpr size_t mfma5_lds_bytes() {
    return (size_t)4 * D * kCT * (NKB * 32 + 16) + kTabCap * 2 + 512;
}

// One pair of tiles (tiles[0], tiles[1]: same item) on the LDS at lds.
template <int NRT, int NKB, int D, int NV, bool Z32>
__device__ static void mfma5_pair(const DevFamily &fam, const DevTile *tp, const DevDigitItem *__restrict__ items,
                                  const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
                                  const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx,
                                  uint64_t *__restrict__ store, uint64_t *__restrict__ hbuf, const uint32_t (&sl)[16],
                                  int *__restrict__ err, int8_t *Xall, const int16_t *colmapL, const int8_t *dirsL) {
    constexpr int K = NKB * 32;
    constexpr int XS = K + 16;
    constexpr int NT = 64 * NRT;
    constexpr int XB = D * kCT * XS;
    (void)K;
    const DevTile tA = tp[0], tB = tp[1];
    const DevDigitItem it = items[tA.item];
    const int s = fam.s, F = fam.F;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 31, half = lane >> 5, bin = 2 * wave + half;
    int8_t *XA = Xall, *XBp = Xall + 2 * XB;  // two plane sets per tile

    v4i A[D][NKB];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int kb = 0; kb < NKB; kb++)
            A[i][kb] = *reinterpret_cast<const v4i *>(it.apack + ((((size_t)wave * D + i) * NKB + kb) * 64 + lane) * 16);
    for (int idx = tid; idx < 4 * XB / 16; idx += NT) reinterpret_cast<v4i *>(Xall)[idx] = v4i{0, 0, 0, 0};
    for (int t = 0; t < 2; t++) {
        const DevTile &tl = t ? tB : tA;
        for (int idx = tid; idx < tl.count * F; idx += NT)
            if (vx[tl.chain0 + idx / F].out < 0) hbuf[(size_t)tl.chain0 * F + idx] = 0;
        for (int idx = tid; idx < tl.count * s; idx += NT) {
            const int out = vx[tl.chain0 + idx / s].out;
            if (out >= 0) store[(size_t)out * s + idx % s] = 0;
        }
    }
    __syncthreads();
    TileState<NV> sA, sB;
    mfma5_init<NRT, NKB, D, NV>(fam, tA, it, cu, cg, cpole, vx, store, err, XA, colmapL, dirsL, sA);
    mfma5_init<NRT, NKB, D, NV>(fam, tB, it, cu, cg, cpole, vx, store, err, XBp, colmapL, dirsL, sB);
    __syncthreads();

    int bad = 0, ca = 0, cb = 0;
    v16i accA[D], accB[D];
    mfma5_products<NKB, D>(A, XA, c, half, accA);
    const int steps = max(tA.steps, tB.steps);
    const int r2 = fam.T - 32 * (NKB - 1);  // target rows in the folded last K-block
    for (int step = 0; step < steps; step++) {
        // phase 1: products of B || finish of A
        mfma5_book<NV>(fam, sA, bad);
        mfma5_phase<NRT, NKB, D, NV, Z32>(A, XBp + cb * XB, c, half, accB, accA, sl, sA, colmapL + sA.dirn * s,
                                          XA + (ca ^ 1) * XB + c * XS, it, XA + ca * XB, tid, r2, bad);
        __syncthreads();
        mfma5_flush<NRT, NKB, D, NV>(fam, sA, XA + (ca ^ 1) * XB, c, bin, tA.chain0, it, store, hbuf, bad);
        mfma5_advance<NV>(sA);
        ca ^= 1;
        // phase 2: products of A (next step) || finish of B
        mfma5_book<NV>(fam, sB, bad);
        mfma5_phase<NRT, NKB, D, NV, Z32>(A, XA + ca * XB, c, half, accA, accB, sl, sB, colmapL + sB.dirn * s,
                                          XBp + (cb ^ 1) * XB + c * XS, it, XBp + cb * XB, tid, r2, bad);
        __syncthreads();
        mfma5_flush<NRT, NKB, D, NV>(fam, sB, XBp + (cb ^ 1) * XB, c, bin, tB.chain0, it, store, hbuf, bad);
        mfma5_advance<NV>(sB);
        cb ^= 1;
    }
    if (bad) atomicOr(err, bad);
    __syncthreads();  // the planes are reused by the next pair
}

template <int NRT, int NKB, int D, int NV, bool Z32>
__global__ __launch_bounds__(64 * NRT) void k_reduce_mfma5(DevFamily fam, const DevDigitItem *__restrict__ items,
                                                           const DevTile *__restrict__ tiles, int npairs,
                                                           int *__restrict__ queue, const int16_t *__restrict__ cu,
                                                           const int32_t *__restrict__ cg,
                                                           const int32_t *__restrict__ cpole,
                                                           const DevVec *__restrict__ vx,
                                                           uint64_t *__restrict__ store, uint64_t *__restrict__ hbuf,
                                                           const uint32_t *__restrict__ slots, int *__restrict__ err) {
    extern __shared__ __align__(16) unsigned char lds5[];
    constexpr int XB = D * kCT * (NKB * 32 + 16);
    int8_t *Xall = reinterpret_cast<int8_t *>(lds5);
    int16_t *colmapL = reinterpret_cast<int16_t *>(lds5 + 4 * XB);
    int8_t *dirsL = reinterpret_cast<int8_t *>(colmapL + kTabCap);
    __shared__ int next;
    uint32_t sl[16];
    mfma4_prologue<NRT, NKB, D, NV, Z32>(fam, slots, sl, colmapL, dirsL);
    if (!queue) {  // one pair per workgroup
        mfma5_pair<NRT, NKB, D, NV, Z32>(fam, tiles + 2 * blockIdx.x, items, cu, cg, cpole, vx, store, hbuf, sl, err,
                                         Xall, colmapL, dirsL);
        return;
    }
    for (;;) {  // persistent: pairs drained through the counter
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        const int pi = next;
        __syncthreads();
        if (pi >= npairs) break;
        mfma5_pair<NRT, NKB, D, NV, Z32>(fam, tiles + 2 * pi, items, cu, cg, cpole, vx, store, hbuf, sl, err, Xall,
                                         colmapL, dirsL);
    }
}

template <int R, int KB, int DD, bool ZZ>
static hipError_t launch_one5(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int npairs,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                              uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int pgrid, int *queue,
                              hipStream_t stream) {
    constexpr size_t lds = mfma5_lds_bytes<R, KB, DD>();
    hipError_t e = hipFuncSetAttribute((const void *)k_reduce_mfma5<R, KB, DD, 3, ZZ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int grid = npairs;
    if (pgrid > 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = std::min(npairs, std::max(1, cus) * pgrid);
    }
    hipLaunchKernelGGL((k_reduce_mfma5<R, KB, DD, 3, ZZ>), dim3(grid), dim3(64 * R), lds, stream, fam, items, tiles,
                       npairs, pgrid > 0 ? queue : nullptr, cu, cg, cpole, vx, store, hbuf, slots, err);
    return hipGetLastError();
}

bool mfma5_supports(const DevFamily &fam, int D);

// tiles: 2 * npairs entries, pair i = (tiles[2i], tiles[2i+1]) of one item
hipError_t launch_reduce_mfma5(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int npairs,
                               const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                               uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int D, bool z32,
                               int pgrid, int *queue, hipStream_t stream);

bool mfma_shape(const DevFamily &fam, int &nrt, int &nkb) {
    nrt = (fam.nsrc + 31) / 32;
    nkb = (fam.T + 31) / 32;
    return ((nrt == 2 && nkb == 2) || (nrt == 3 && nkb == 3)) && fam.ndir * fam.s <= kTabCap &&
           fam.s * fam.nv <= kGCap && fam.nv <= 8;
}

template <int R, int KB, int DD, bool ZZ>
static hipError_t launch_one4(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                              uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int pgrid, int *queue,
                              hipStream_t stream) {
    if (pgrid > 0) {
        // resident workgroups per CU of this instance, times the CU count, times pgrid
        static int per_device = 0;
        if (per_device == 0) {
            int dev = 0, cus = 0, per_cu = 0;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_reduce_mfma4_persistent<R, KB, DD, 3, ZZ>,
                                                               64 * R, 0);
            per_device = std::max(1, cus) * std::max(1, per_cu);
        }
        const int grid = std::min(ntiles, per_device * pgrid);
        hipLaunchKernelGGL((k_reduce_mfma4_persistent<R, KB, DD, 3, ZZ>), dim3(grid), dim3(64 * R), 0, stream, fam,
                           items, tiles, ntiles, queue, cu, cg, cpole, vx, store, hbuf, slots, err);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_reduce_mfma4<R, KB, DD, 3, ZZ>), dim3(ntiles), dim3(64 * R), 0, stream, fam, items, tiles, cu,
                       cg, cpole, vx, store, hbuf, slots, err);
    return hipGetLastError();
}

// Shape of the register-gather kernel: up to 64 source rows in 2 row tiles
// (2 waves), up to 128 in 4 (4 waves: every SIMD of the CU gets one wave and
// the outputs spread over 8 lane bins).
bool mfma4_shape(const DevFamily &fam, int &nrt, int &nkb) {
    nrt = fam.nsrc <= 64 ? 2 : (fam.nsrc <= 128 ? 4 : 0);
    nkb = (fam.T + 31) / 32;
    return nrt > 0 && ((nrt == 2 && nkb == 2) || (nrt == 4 && nkb == 3)) && fam.ndir * fam.s <= kTabCap &&
           fam.nv <= 8;
}

bool mfma4_supports(const DevFamily &fam, int D) {
    int nrt, nkb;
    if (!mfma4_shape(fam, nrt, nkb) || fam.nv != 3 || fam.ndir * fam.nv > 512) return false;
    return (nrt == 2 && (D == 3 || D == 6)) || (nrt == 4 && (D == 5 || D == 8 || D == 10));
}

hipError_t launch_reduce_mfma4(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                               const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                               uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int D, bool z32,
                               int pgrid, int *queue, hipStream_t stream) {
    if (ntiles == 0) return hipSuccess;
    int nrt, nkb;
    if (!mfma4_supports(fam, D)) return hipErrorInvalidValue;
    mfma4_shape(fam, nrt, nkb);
#define CRF_LAUNCH4(R, KB, DD)                                                                                          \
    if (nrt == R && nkb == KB && D == DD) {                                                                             \
        if (z32)                                                                                                        \
            return launch_one4<R, KB, DD, true>(fam, items, tiles, ntiles, cu, cg, cpole, vx, store, hbuf, slots, err,  \
                                                pgrid, queue, stream);                                                  \
        return launch_one4<R, KB, DD, false>(fam, items, tiles, ntiles, cu, cg, cpole, vx, store, hbuf, slots, err,     \
                                             pgrid, queue, stream);                                                     \
    }
    CRF_LAUNCH4(2, 2, 3)
    CRF_LAUNCH4(2, 2, 6)
    CRF_LAUNCH4(4, 3, 5)
    CRF_LAUNCH4(4, 3, 8)
    CRF_LAUNCH4(4, 3, 10)
#undef CRF_LAUNCH4
    return hipErrorInvalidValue;
}

bool mfma5_supports(const DevFamily &fam, int D) {
    int nrt, nkb;
    if (!mfma4_supports(fam, D)) return false;
    mfma4_shape(fam, nrt, nkb);
    // the last K-block is folded: its R2 target rows times D digits fit one block
    const int r2 = fam.T - 32 * (nkb - 1);
    if (r2 < 1 || r2 * D > 32) return false;
    if (fam.s > 32 * (nkb - 1)) return false;  // parked digits stay below the folded block
    // the digits of an ending chain are parked at columns r < s of its rows
    if (fam.s > nkb * 32) return false;
    // the two tiles' accumulators (2 D x 16 registers) must fit the 256 AGPRs:
    // D = 10 (plane quintics at p = 17 .. 29) would spill them to scratch
    return (nrt == 4 && (D == 5 || D == 8)) || (nrt == 2 && (D == 3 || D == 6));
}

hipError_t launch_reduce_mfma5(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int npairs,
                               const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                               uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int D, bool z32,
                               int pgrid, int *queue, hipStream_t stream) {
    if (npairs == 0) return hipSuccess;
    int nrt, nkb;
    if (!mfma5_supports(fam, D)) return hipErrorInvalidValue;
    mfma4_shape(fam, nrt, nkb);
#define CRF_LAUNCH5(R, KB, DD)                                                                                      \
    if (nrt == R && nkb == KB && D == DD) {                                                                         \
        if (z32)                                                                                                    \
            return launch_one5<R, KB, DD, true>(fam, items, tiles, npairs, cu, cg, cpole, vx, store, hbuf, slots,   \
                                                err, pgrid, queue, stream);                                         \
        return launch_one5<R, KB, DD, false>(fam, items, tiles, npairs, cu, cg, cpole, vx, store, hbuf, slots, err, \
                                             pgrid, queue, stream);                                                 \
    }
    CRF_LAUNCH5(2, 2, 3)
    CRF_LAUNCH5(2, 2, 6)
    CRF_LAUNCH5(4, 3, 5)
    CRF_LAUNCH5(4, 3, 8)
#undef CRF_LAUNCH5
    return hipErrorInvalidValue;
}

bool mfma_supports_digits(int D) { return D == 3 || D == 5 || D == 6 || D == 8 || D == 10; }

template <int R, int KB, int DD>
static hipError_t launch_one(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                             const int16_t *cu, const int32_t *cg, const int32_t *cpole, uint64_t *hbuf, int *err,
                             hipStream_t stream) {
    const size_t lds = mfma_lds_bytes_rt(KB, DD, fam.nsrc);
    hipError_t e = hipFuncSetAttribute((const void *)k_reduce_mfma<R, KB, DD>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reduce_mfma<R, KB, DD>), dim3(ntiles), dim3(64 * R), lds, stream, fam, items, tiles, cu, cg,
                       cpole, hbuf, err);
    return hipGetLastError();
}

hipError_t launch_reduce_mfma(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, uint64_t *hbuf, int *err,
                              int D, hipStream_t stream) {
    if (ntiles == 0) return hipSuccess;
    int nrt, nkb;
    if (!mfma_shape(fam, nrt, nkb)) return hipErrorInvalidValue;
#define CRF_LAUNCH(R, KB, DD) \
    if (nrt == R && nkb == KB && D == DD) return launch_one<R, KB, DD>(fam, items, tiles, ntiles, cu, cg, cpole, hbuf, err, stream);
    CRF_LAUNCH(2, 2, 3)
    CRF_LAUNCH(2, 2, 5)
    CRF_LAUNCH(2, 2, 6)
    CRF_LAUNCH(2, 2, 8)
    CRF_LAUNCH(2, 2, 10)
    CRF_LAUNCH(3, 3, 3)
    CRF_LAUNCH(3, 3, 5)
    CRF_LAUNCH(3, 3, 6)
    CRF_LAUNCH(3, 3, 8)
    CRF_LAUNCH(3, 3, 10)
#undef CRF_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace crf
