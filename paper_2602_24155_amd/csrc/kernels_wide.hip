// Exact int8-digit MFMA reduction for families whose right inverse and
// digit planes do not stay on chip: cubic threefolds (five variables, degree
// 3, S = {x_4}: s = 495 outputs, J_S from 1815 source to 1001 target rows;
// Definition 3.1 and Proposition 3.3 with S a proper subset) and quintic
// surfaces (four variables, degree 5, S = all: s = 455, J_S from 880 source
// to 560 target rows).
//
// The step is the one of the quad kernel (kernels_quad.hip): for 32 vectors
// of one hypersurface
//   t  = psi[:, cols(v)] w                                  (nsrc values)
//   w'[r] = sum_i (u_i + r_i + [i not in S]) t[src(r, i)]   (s values)
// with t one integer product on the matrix cores over balanced base-B digits
// (B = p^e <= 169, Q' = B^D) and the gather on the accumulators.  What
// differs is the size: 57 row tiles of psi and 32 K-blocks for threefolds, 28
// and 18 for quintic surfaces, so neither psi's digits nor the vectors' digit
// planes (D x 32 x (32 K + 16) bytes per set, more than the LDS holds for
// two sets) stay on chip.  Each workgroup keeps its two plane sets in a slice
// of global memory (L2-resident; only the family tables are in LDS) and every
// wave takes its row tiles two at a time, streaming psi's digit fragments of
// both and the planes' fragments once for the two, one K-block ahead.  All
// waves of a workgroup run on one CU, so the workgroup barrier orders their
// writes and reads of the planes as it does for LDS.
//
// Row placement.  Threefolds ("quint" tiles): an output with r_4 >= 1 has
// five source rows, one per variable; one with r_4 = 0 has only the row of
// x_4.  The host places, in each lane half's 16 accumulator rows of the first
// row tiles, three five-source outputs (slots 5 q + i, variable i) and one
// one-source output (slot 15); the last row tiles hold sixteen one-source
// outputs per lane half.  330 five-source and 165 one-source outputs fill 55
// + 2 row tiles (1815 of 1824 rows).  Quintic surfaces (the quad placement of
// the K3 kernel): an output with every r_i >= 1 has four source rows, one
// with a single r_z = 0 only the row of x_z; 165 four-source outputs fill 21
// quad row tiles (four per lane half, slots 4 q + i), the 4 x 55 one-source
// outputs 7 more (slot 4 q + t of variable t): 880 of 896 rows.
//
// The carry step is the quad kernel's: t = z_k + carry, carry = round(t / B)
// in fp64 (|t| < 2^48, checked on the host), digit = t - B carry.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_layout.hpp"

namespace crf {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(1))) v4i gv4i;

constexpr int kWV = 32;       // vectors per tile
constexpr int kWWaves = 4;    // waves per workgroup
constexpr int kWTab = 25600;  // colmap entries (ndir x s) held in LDS
constexpr int kWSmall = 256;  // bytes for the direction and final-exponent tables

template <int NRT, int NKB, int D>
struct WideShape {
    static constexpr int K = NKB * 32;
    static constexpr int XS = K + 16;          // bytes per (digit, vector) row of the planes
    static constexpr int XB = D * kWV * XS;    // one set of digit planes (global memory)
    static constexpr size_t lds = (size_t)kWTab * 2 + 2 * kWSmall + (size_t)NRT * 2 * 16 * 4;
};

// Algorithm 3 for S given by smask: one unit on every variable of S with
// u_i != 0, then one unit at a time, round robin over all variables, while
// v_i < u_i; k = the largest chunk with u - k v >= 0, capped by the pole
// orders left; dir = index of v in the direction table (-1 if none).
template <int NV>
__device__ __forceinline__ void choose_chunk_w(int d, uint32_t smask, int ndir, const int8_t *dirsL, const int *U,
                                               int poles_left, int *v, int &dir, int &k) {
    int left = d;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        v[i] = (left > 0 && ((smask >> i) & 1u) && U[i] != 0) ? 1 : 0;
        left -= v[i];
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
    if (left == 0)
        for (int t = 0; t < ndir && dir < 0; t++) {
            bool eq = true;
#pragma unroll
            for (int i = 0; i < NV; i++) eq = eq && dirsL[NV * t + i] == v[i];
            if (eq) dir = t;
        }
}

// Balanced base-B digits of x in [0, q) (q | Q'), written D planes apart
// (v < Q' < 2^52, exact in fp64; the quotient from the product with 1 / B is
// off by at most one).
template <int D, int XS>
__device__ __forceinline__ void put_digits_w(int8_t *xp, uint64_t x, uint64_t Qp, int B, double invB, int halfB) {
    uint64_t v = x + (Qp - 1) / 2;
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
        xp[k * kWV * XS] = (int8_t)((int)r - halfB);
        v = qd;
    }
}

// Output r of a vector from its weighted position sums: carry propagation to
// balanced digits, then the digits of the next step, or the value mod q
// (combine store or pole-n numerators).
template <int D, int XS>
__device__ __forceinline__ void emit_w(const double (&z)[D], int r, bool more, const int16_t *cm, int8_t *Xn_c,
                                       int vout, int fin_row, const int16_t *__restrict__ finmap, uint64_t *hrow,
                                       uint64_t *__restrict__ store, int s, double Bd, double invB, int64_t Bi,
                                       int64_t q, double invq, int &bad) {
    int dg[D];
    double carry = 0.0;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const double t = z[k] + carry;
        const double cq = rint(t * invB);
        dg[k] = (int)fma(-cq, Bd, t);
        carry = cq;
    }
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
        for (int k = 0; k < D; k++) Xn_c[k * kWV * XS + col] = (int8_t)dg[k];
        return;
    }
    int64_t x = 0;
#pragma unroll
    for (int k = D - 1; k >= 0; k--) x = x * Bi + dg[k];
    // |x| < Q' / 2 < 2^51: the floored quotient by q from fp64 is off by at most one
    x -= (int64_t)floor((double)x * invq) * q;
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

template <int D, int NKB>
__device__ __forceinline__ void load_a(const int8_t *base, int rt, int kb, v4i (&dst)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) dst[i] = *(gv4i *)(base + (((size_t)rt * D + i) * NKB + kb) * 1024);
}

template <int D, int XS>
__device__ __forceinline__ void load_x(const int8_t *xc, int kb, v4i (&dst)[D]) {
#pragma unroll
    for (int j = 0; j < D; j++) dst[j] = *(gv4i *)(xc + (size_t)j * kWV * XS + kb * 32);
}

template <int D>
__device__ __forceinline__ void products(const v4i (&a)[D], const v4i (&x)[D], v16i (&acc)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; i + j < D; j++)
            acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], x[j], acc[i + j], 0, 0, 0);
}

// Products of row tiles rt and (TWO) rt2 with the current planes over all
// K-blocks, in pairs of K-blocks with two fragment buffers: the loads of the
// next block are in flight during the products of this one.
template <int D, int NKB, int XS, bool TWO>
__device__ __forceinline__ void pair_products(const int8_t *abase, const int8_t *xbase, int rt, int rt2,
                                              v16i (&acc)[D], v16i (&acc2)[D]) {
    v4i a0[D], b0[D], x0[D], a1[D], b1[D], x1[D];
    load_a<D, NKB>(abase, rt, 0, a0);
    if (TWO) load_a<D, NKB>(abase, rt2, 0, b0);
    load_x<D, XS>(xbase, 0, x0);
    for (int kb = 0; kb < NKB; kb += 2) {
        load_a<D, NKB>(abase, rt, kb + 1, a1);
        if (TWO) load_a<D, NKB>(abase, rt2, kb + 1, b1);
        load_x<D, XS>(xbase, kb + 1, x1);
        products<D>(a0, x0, acc);
        if (TWO) products<D>(b0, x0, acc2);
        if (kb + 2 < NKB) {
            load_a<D, NKB>(abase, rt, kb + 2, a0);
            if (TWO) load_a<D, NKB>(abase, rt2, kb + 2, b0);
            load_x<D, XS>(xbase, kb + 2, x0);
        }
        products<D>(a1, x1, acc);
        if (TWO) products<D>(b1, x1, acc2);
    }
}

// The outputs of row tile rt held by this lane half.  Five variables (quint
// tiles): three five-source outputs (slots 5 qd + i, variable i) and one
// one-source output (slot 15), past the quint tiles sixteen one-source
// outputs.  Four variables (quad tiles): four four-source outputs (slots
// 4 qd + i, variable i), past the quad tiles sixteen one-source outputs
// (slot 4 qd + t of variable t).  NRTQ: the number of quint or quad tiles.
template <int NV, int NRTQ, int D, int XS>
__device__ __forceinline__ void finish_rt(int rt, int half, const v16i (&acc)[D], const uint32_t *slotL,
                                          const int (&up)[NV], bool more, const int16_t *cm, int8_t *Xn_c, int vout,
                                          int fin_row, const int16_t *__restrict__ finmap, uint64_t *hrow,
                                          uint64_t *__restrict__ store, int s, double Bd, double invB, int64_t Bi,
                                          int64_t q, double invq, int &bad) {
    constexpr int NG = NV == 5 ? 3 : 4;  // multi-source outputs per lane half of a quint / quad tile
    const uint32_t *sb = slotL + (rt * 2 + half) * 16;
    if (rt < NRTQ) {
#pragma unroll
        for (int qd = 0; qd < NG; qd++) {
            const uint32_t w0 = sb[NV * qd];
            const int r = (int)(w0 >> 16);
            if (r == 0xFFFF) continue;
            double z[D];
#pragma unroll
            for (int k = 0; k < D; k++) z[k] = 0.0;
#pragma unroll
            for (int t = 0; t < NV; t++) {
                const double wt = (double)(up[t] + (int)((sb[NV * qd + t] >> 5) & 2047u));
#pragma unroll
                for (int k = 0; k < D; k++) z[k] = fma(wt, (double)acc[k][NV * qd + t], z[k]);
            }
            emit_w<D, XS>(z, r, more, cm, Xn_c, vout, fin_row, finmap, hrow, store, s, Bd, invB, Bi, q, invq, bad);
        }
        if constexpr (NV == 5) {
            const uint32_t w = sb[15];
            if (w & 1u) {
                const int iv = (int)((w >> 2) & 7u);
                const double wt = (double)(up[iv] + (int)((w >> 5) & 2047u));
                double z[D];
#pragma unroll
                for (int k = 0; k < D; k++) z[k] = wt * (double)acc[k][15];
                emit_w<D, XS>(z, (int)(w >> 16), more, cm, Xn_c, vout, fin_row, finmap, hrow, store, s, Bd, invB, Bi,
                              q, invq, bad);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const uint32_t w = sb[j];
            if (!(w & 1u)) continue;
            const int iv = (int)((w >> 2) & 7u);
            const double wt = (double)(up[iv] + (int)((w >> 5) & 2047u));
            double z[D];
#pragma unroll
            for (int k = 0; k < D; k++) z[k] = wt * (double)acc[k][j];
            emit_w<D, XS>(z, (int)(w >> 16), more, cm, Xn_c, vout, fin_row, finmap, hrow, store, s, Bd, invB, Bi, q,
                          invq, bad);
        }
    }
}

// One tile (up to 32 vectors of one item) on the workgroup's plane sets X
// (global memory, 2 XB bytes).
template <int NV, int NRT, int NRTQ, int NKB, int D>
__device__ void wide_tile(const DevFamily &fam, const DevTile &tile, const DevDigitItem *__restrict__ items,
                          const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
                          const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx,
                          uint64_t *__restrict__ store, uint64_t *__restrict__ hbuf, int &bad, int8_t *X,
                          const int16_t *colmapL, const int8_t *dirsL, const int8_t *finUL, const uint32_t *slotL) {
    using Sh = WideShape<NRT, NKB, D>;
    constexpr int XS = Sh::XS, XB = Sh::XB, NT = 64 * kWWaves;
    const int s = fam.s, F = fam.F;
    const DevDigitItem it = items[tile.item];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int c = lane & 31, half = lane >> 5;
    const int nch = tile.count;

    for (int idx = tid; idx < 2 * XB / 16; idx += NT) reinterpret_cast<v4i *>(X)[idx] = v4i{0, 0, 0, 0};
    for (int cc = 0; cc < nch; cc++) {
        const int out = vx[tile.chain0 + cc].out;
        if (out < 0)
            for (int e = tid; e < F; e += NT) hbuf[(size_t)(tile.chain0 + cc) * F + e] = 0;
        else
            for (int e = tid; e < s; e += NT) store[(size_t)out * s + e] = 0;
    }
    __syncthreads();

    const double Bd = it.Bd, invB = 1.0 / it.Bd;
    const int64_t Bi = it.B, q = (int64_t)it.q;
    const double invq = 1.0 / (double)it.q;

    int U[NV] = {}, V[NV] = {};
    int dir = 0, kleft = 0, pole = fam.n, pend = fam.n, vout = -1;
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
            choose_chunk_w<NV>(fam.d, fam.smask, fam.ndir, dirsL, U, pole - pend, V, d0, k0);
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
                else X[c * XS + col] = (int8_t)1;  // balanced digits of 1
            }
        } else {
            // start vector from the combine store: the 8 lanes of vector c split its entries
            for (int r = 2 * wave + half; r < s; r += 2 * kWWaves) {
                const uint64_t x = store[(size_t)xv.in * s + r];
                if (x == 0) continue;
                const int col = colmapL[d0 * s + r];
                if (col < 0) {
                    bad |= 2;
                    continue;
                }
                put_digits_w<D, XS>(X + c * XS + col, x, it.Qp, it.B, invB, it.halfB);
            }
        }
    }
    __syncthreads();

    int cur = 0;
    for (int step = 0; step < tile.steps; step++) {
        const int8_t *Xc = X + cur * XB;
        int8_t *Xn = X + (cur ^ 1) * XB;
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
            choose_chunk_w<NV>(fam.d, fam.smask, fam.ndir, dirsL, up, pole - 1 - pend, Vn, d0, k0);
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
            for (int a = 0; a < fam.nfinU && Ui < 0; a++) {
                bool eq = true;
#pragma unroll
                for (int i = 0; i < NV; i++) eq = eq && finUL[NV * a + i] == up[i];
                if (eq) Ui = a;
            }
            if (Ui < 0) bad |= 4;
            else fin_row = Ui * s;
        }
        const int16_t *cm = colmapL + dirn * s;
        int8_t *Xn_c = Xn + c * XS;
        uint64_t *hrow = hbuf + (size_t)(tile.chain0 + c) * F;

        const int8_t *abase = it.apack + lane * 16;
        const int8_t *xbase = Xc + c * XS + half * 16;
        // row tiles in pairs (rt, rt + 4): one stream of the planes' fragments
        // feeds the products of both, which halves the plane reads
        for (int rt = wave; rt < NRT; rt += 2 * kWWaves) {
            const int rt2 = rt + kWWaves;
            v16i acc[D], acc2[D];
#pragma unroll
            for (int k = 0; k < D; k++) acc[k] = acc2[k] = v16i{0};
            if (rt2 < NRT)
                pair_products<D, NKB, XS, true>(abase, xbase, rt, rt2, acc, acc2);
            else
                pair_products<D, NKB, XS, false>(abase, xbase, rt, rt, acc, acc2);
            if (!act) continue;
            finish_rt<NV, NRTQ, D, XS>(rt, half, acc, slotL, up, more, cm, Xn_c, vout, fin_row, fam.finmap, hrow, store, s,
                                   Bd, invB, Bi, q, invq, bad);
            if (rt2 < NRT)
                finish_rt<NV, NRTQ, D, XS>(rt2, half, acc2, slotL, up, more, cm, Xn_c, vout, fin_row, fam.finmap, hrow,
                                       store, s, Bd, invB, Bi, q, invq, bad);
        }
        __syncthreads();  // every wave has read the current planes and written the next ones
        int8_t *Xz = X + cur * XB;
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
        __syncthreads();  // the cleared planes are free for the next step's digits
    }
}

// A persistent grid draining the tile list through the counter *queue (zero
// at launch; every workgroup leaves once the counter passes ntiles).
// Workgroup b works on the plane sets at xscratch + 2 XB b.
template <int NV, int NRT, int NRTQ, int NKB, int D>
__global__ __launch_bounds__(64 * kWWaves) void k_reduce_wide(
    DevFamily fam, const DevDigitItem *__restrict__ items, const DevTile *__restrict__ tiles, int ntiles,
    int *__restrict__ queue, const int16_t *__restrict__ cu, const int32_t *__restrict__ cg,
    const int32_t *__restrict__ cpole, const DevVec *__restrict__ vx, uint64_t *__restrict__ store,
    uint64_t *__restrict__ hbuf, const uint32_t *__restrict__ slots, int8_t *__restrict__ xscratch,
    int *__restrict__ err) {
    using Sh = WideShape<NRT, NKB, D>;
    extern __shared__ __align__(16) unsigned char ldsw[];
    int16_t *colmapL = reinterpret_cast<int16_t *>(ldsw);
    int8_t *dirsL = reinterpret_cast<int8_t *>(colmapL + kWTab);
    int8_t *finUL = dirsL + kWSmall;
    uint32_t *slotL = reinterpret_cast<uint32_t *>(finUL + kWSmall);
    __shared__ int next;
    const int NT = 64 * kWWaves, tid = threadIdx.x;
    for (int idx = tid; idx < fam.ndir * fam.s; idx += NT) colmapL[idx] = fam.colmap[idx];
    for (int idx = tid; idx < fam.ndir * NV; idx += NT) dirsL[idx] = fam.dirs[idx];
    for (int idx = tid; idx < fam.nfinU * NV; idx += NT) finUL[idx] = fam.finU[idx];
    for (int idx = tid; idx < NRT * 2 * 16; idx += NT) slotL[idx] = slots[idx];
    int8_t *X = xscratch + (size_t)blockIdx.x * 2 * Sh::XB;
    int bad = 0;
    for (;;) {
        if (tid == 0) next = atomicAdd(queue, 1);
        __syncthreads();  // also publishes the tables before the first tile
        const int ti = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();  // every thread has read `next` before it is overwritten
        if (ti >= ntiles) break;
        wide_tile<NV, NRT, NRTQ, NKB, D>(fam, tiles[ti], items, cu, cg, cpole, vx, store, hbuf, bad, X, colmapL, dirsL,
                                     finUL, slotL);
    }
    if (bad) atomicOr(err, bad);
}

template <int NV, int NRT, int NRTQ, int NKB, int D>
hipError_t launch_wide_one(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                           const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                           uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int8_t *xscratch, int grid,
                           int *err, int *queue, hipStream_t stream) {
    constexpr size_t lds = WideShape<NRT, NKB, D>::lds;
    hipError_t e = hipFuncSetAttribute((const void *)k_reduce_wide<NV, NRT, NRTQ, NKB, D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reduce_wide<NV, NRT, NRTQ, NKB, D>), dim3(grid), dim3(64 * kWWaves), lds, stream, fam,
                       items, tiles, ntiles, queue, cu, cg, cpole, vx, store, hbuf, slots, xscratch, err);
    return hipGetLastError();
}

}  // namespace

// Shape of the streaming kernel for a family: cubic threefolds (five
// variables, S = {x_4}): 57 row tiles, the first 55 quint tiles, 32
// K-blocks; quintic surfaces (four variables, S = all): 28 row tiles, the
// first 21 quad tiles, 18 K-blocks.
bool wide_shape(const DevFamily &fam, int &nrt, int &nrtq, int &nkb) {
    const bool tables = fam.ndir * fam.s <= kWTab && fam.ndir * fam.nv <= kWSmall && fam.nfinU * fam.nv <= kWSmall;
    if (fam.nv == 5 && fam.smask == 0x10u && fam.s == 495 && fam.T == 1001 && fam.nsrc == 1815) {
        nrt = 57;
        nrtq = 55;
        nkb = 32;
        return tables;
    }
    if (fam.nv == 4 && fam.smask == 0xFu && fam.s == 455 && fam.T == 560 && fam.nsrc == 880) {
        nrt = 28;
        nrtq = 21;
        nkb = 18;
        return tables;
    }
    return false;
}

bool wide_supports_digits(int D) { return D >= 4 && D <= 7; }

// Bytes of global memory for the digit planes of `grid` workgroups.
size_t wide_scratch_bytes(int D, int grid) { return (size_t)grid * 2 * D * kWV * (32 * 32 + 16); }

// Workgroups of the persistent launch: pgrid per CU, at most one per tile.
int wide_grid(int ntiles, int pgrid) {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return std::max(1, std::min(ntiles, std::max(1, cus) * std::max(1, pgrid)));
}

// One persistent launch for the tiles of items with D digits; xscratch holds
// wide_scratch_bytes(D, grid) bytes.
hipError_t launch_reduce_wide(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                              uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int D, int grid,
                              int8_t *xscratch, int *queue, hipStream_t stream) {
    if (ntiles == 0) return hipSuccess;
    int nrt, nrtq, nkb;
    if (!wide_shape(fam, nrt, nrtq, nkb) || !wide_supports_digits(D) || !queue) return hipErrorInvalidValue;
#define CRF_WIDE(NV, R, RQ, KB, DD)                                                                              \
    return launch_wide_one<NV, R, RQ, KB, DD>(fam, items, tiles, ntiles, cu, cg, cpole, vx, store, hbuf, slots,       \
                                              xscratch, grid, err, queue, stream)
    if (nrt == 57) {
        switch (D) {
            case 4: CRF_WIDE(5, 57, 55, 32, 4);
            case 5: CRF_WIDE(5, 57, 55, 32, 5);
            case 6: CRF_WIDE(5, 57, 55, 32, 6);
            default: CRF_WIDE(5, 57, 55, 32, 7);
        }
    }
    switch (D) {
        case 4: CRF_WIDE(4, 28, 21, 18, 4);
        case 5: CRF_WIDE(4, 28, 21, 18, 5);
        case 6: CRF_WIDE(4, 28, 21, 18, 6);
        default: CRF_WIDE(4, 28, 21, 18, 7);
    }
#undef CRF_WIDE
}

}  // namespace crf
