// Right inverse psi of J_S mod q = p^M on the device, and its int8 digits
// for the MFMA reduction kernel (gfx950).  One launch covers every
// hypersurface of a call: it needs only the coefficients of f.
//
// psi is the decomposition map of Proposition 3.3: for a numerator h in the
// target of J_S, psi h gives the g_i with h = sum_{i in S} g_i d_i f +
// sum_{i not in S} g_i x_i d_i f.  One workgroup per hypersurface runs
// Gauss-Jordan elimination on [J | I] (R = dim target rows, C = nsrc source
// columns) in LDS: row r takes as pivot the first unused column whose entry is
// a unit mod p (so every pivot is invertible mod p^M), scales the row by the
// pivot's inverse (Fermat mod p, then Newton lifting y <- y (2 - a y) to
// p^M) and clears the pivot column in every other row.  psi[c_r, :] is then
// row r of the right half, and psi is zero on the non-pivot source rows.
// A row without a unit pivot means J_S is not surjective mod p (f is not
// S-smooth): the item's flag is set and its psi is left zero.
#include <hip/hip_runtime.h>

#include "device_layout.hpp"

namespace crf {

typedef unsigned __int128 u128p;

struct PMod {
    uint64_t q, mu;
    int sbits;
    __device__ __forceinline__ uint64_t reduce(u128p x) const {  // x < 2^(2 sbits + 8)
        const uint64_t x1 = (uint64_t)(x >> (sbits - 1));
        const uint64_t qh = (uint64_t)(((u128p)x1 * mu) >> (sbits + 9));
        uint64_t r = (uint64_t)x - qh * q;
        r = r >= q ? r - q : r;
        r = r >= q ? r - q : r;
        return r;
    }
    __device__ __forceinline__ uint64_t mul(uint64_t a, uint64_t b) const { return reduce((u128p)a * b); }
};

// x mod p for a small p with 32-bit operations: x = hi 2^32 + lo
__device__ __forceinline__ static uint32_t mod_small(uint64_t x, uint32_t p, uint32_t two32p) {
    const uint32_t hi = (uint32_t)(x >> 32) % p, lo = (uint32_t)x % p;
    return (hi * two32p + lo) % p;
}

// inverse of a unit a mod q = p^M
__device__ static uint64_t inv_mod(const PMod &md, uint64_t a, uint32_t p, uint32_t two32p) {
    const uint32_t a0 = mod_small(a, p, two32p);
    uint32_t y0 = 1, base = a0, e = p - 2;  // a0^(p-2) mod p
    while (e) {
        if (e & 1) y0 = (y0 * base) % p;
        base = (base * base) % p;
        e >>= 1;
    }
    uint64_t y = y0;
    // each step doubles the number of correct p-adic digits (7 steps reach p^128)
    for (int it = 0; it < 7; it++) {
        const uint64_t ay = md.mul(a, y);
        const uint64_t t = ay <= 2 ? 2 - ay : 2 + md.q - ay;  // 2 - a y mod q
        const uint64_t y2 = md.mul(y, t);
        if (y2 == y) break;
        y = y2;
    }
    return y;
}

// 16 waves per workgroup (4 per SIMD): the elimination is bound by the
// latency of its LDS reads and 64-bit products, which the extra waves hide
constexpr int kPsiThreads = 1024;
constexpr int kPsiWaves = kPsiThreads / 64;

// LDS: [J | I] (R x (C + R) u64), the pivot column snapshot (R u64), the
// pivot inverse (u64), the pivot marks of the columns (C int), 8 int of scratch
size_t psi_lds_bytes(int R, int C) { return (size_t)R * (C + R) * 8 + (size_t)(R + 1) * 8 + (size_t)C * 4 + 32; }

// LDS of the global-memory form: everything but [J | I]
size_t psi_small_lds_bytes(int R, int C) { return (size_t)(R + 1) * 8 + (size_t)C * 4 + 32; }

// bytes of one item's bookkeeping in the device-wide elimination (16-byte aligned)
__host__ __device__ inline size_t gj_book_bytes(int R, int C) {
    return ((size_t)(R + 1) * 8 + (size_t)(C + 2) * 4 + 15) / 16 * 16;
}

// J_S is built from the coefficients of f and the family table jtab: entry
// (r, k) = c_e * w for jtab[r C + k] = (e << 8) | w, or 0 for -1.  `a` holds
// [J | I] (R x (C + R)), in LDS (k_psi) or in global memory (k_psi_global,
// for families whose matrix does not fit the LDS); the pivot bookkeeping is
// in LDS either way.
__device__ static void psi_eliminate(const DevItem &it, int R, int C, const int32_t *__restrict__ jtab, uint64_t *a,
                                     unsigned char *small) {
    const PMod md{it.q, it.mu, it.sbits};
    const uint32_t p = (uint32_t)it.p, two32p = (uint32_t)((1ull << 32) % p);
    const int W = C + R, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *fcol = reinterpret_cast<uint64_t *>(small);
    uint64_t *shinv = fcol + R;
    int *used = reinterpret_cast<int *>(shinv + 1);
    int *sh = used + C;  // sh[0]: pivot column, sh[1]: failure
    for (int r = wave; r < R; r += kPsiWaves)
        for (int k = lane; k < W; k += 64)
            if (k < C) {
                const int32_t e = jtab[(size_t)r * C + k];
                a[(size_t)r * W + k] = e < 0 ? 0 : md.reduce((u128p)it.fcoef[e >> 8] * (uint32_t)(e & 255));
            } else {
                a[(size_t)r * W + k] = (uint64_t)(k - C == r);
            }
    for (int k = tid; k < C; k += kPsiThreads) used[k] = 0;
    if (tid == 0) sh[1] = 0;
    __syncthreads();
    for (int r = 0; r < R; r++) {
        uint64_t *row = a + (size_t)r * W;
        if (wave == 0) {
            // first unused column holding a unit mod p (columns k = lane + 64 j)
            int c = C;
            for (int k0 = 0; k0 < C && c == C; k0 += 64) {
                const int k = k0 + lane;
                const bool ok = k < C && !used[k] && mod_small(row[k], p, two32p) != 0;
                const unsigned long long m = __ballot(ok);
                if (m) c = k0 + __ffsll((long long)m) - 1;
            }
            if (lane == 0) {
                sh[0] = c;
                if (c == C) sh[1] = 1;
                else shinv[0] = inv_mod(md, row[c], p, two32p);
            }
        }
        __syncthreads();
        const int c = sh[0];
        if (c == C) break;  // uniform: every thread read the same sh[0]
        const uint64_t inv = shinv[0];
        for (int k = tid; k < W; k += kPsiThreads) row[k] = md.mul(row[k], inv);
        for (int r2 = tid; r2 < R; r2 += kPsiThreads) fcol[r2] = r2 == r ? 0 : a[(size_t)r2 * W + c];
        __syncthreads();
        // clear column c: each wave takes whole rows, skipping those already zero there
        for (int r2 = wave; r2 < R; r2 += kPsiWaves) {
            const uint64_t f = fcol[r2];
            if (f == 0) continue;
            uint64_t *o = a + (size_t)r2 * W;
            for (int k = lane; k < W; k += 64) {
                const uint64_t t = md.mul(f, row[k]);
                const uint64_t x = o[k];
                o[k] = x >= t ? x - t : x + md.q - t;
            }
        }
        if (tid == 0) used[c] = r + 1;  // pivot of row r (1-based)
        __syncthreads();
    }
    const bool fail = sh[1] != 0;
    if (tid == 0 && fail) atomicOr(it.flag, 1);
    // psi (C x R): row c = pivot of row r -> right half of row r
    for (int cc = wave; cc < C; cc += kPsiWaves) {
        const int r1 = used[cc];
        for (int j = lane; j < R; j += 64)
            it.psi_out[(size_t)cc * R + j] = (!fail && r1 > 0) ? a[(size_t)(r1 - 1) * W + C + j] : 0;
    }
}

// An item with q = 0 (rejected on the host) is skipped.
__global__ __launch_bounds__(kPsiThreads) void k_psi(const DevItem *__restrict__ items, int R, int C,
                                                     const int32_t *__restrict__ jtab) {
    extern __shared__ __align__(16) unsigned char lds[];
    const DevItem it = items[blockIdx.x];
    if (it.q == 0) return;  // uniform over the workgroup
    uint64_t *a = reinterpret_cast<uint64_t *>(lds);
    psi_eliminate(it, R, C, jtab, a, reinterpret_cast<unsigned char *>(a + (size_t)R * (C + R)));
}

// [J | I] of item i at work + i R (C + R) (global memory: 978 KB for quartic
// K3 surfaces).  All of a workgroup's waves run on one CU, so its barriers
// order their global reads and writes as they do for LDS.
__global__ __launch_bounds__(kPsiThreads) void k_psi_global(const DevItem *__restrict__ items, int R, int C,
                                                            const int32_t *__restrict__ jtab, uint64_t *work) {
    extern __shared__ __align__(16) unsigned char lds[];
    const DevItem it = items[blockIdx.x];
    if (it.q == 0) return;
    psi_eliminate(it, R, C, jtab, work + (size_t)blockIdx.x * R * (C + R), lds);
}

// Balanced base-B digits of psi in v_mfma_i32_32x32x32_i8 A-fragment order,
// source rows placed by the bin layout:
// apack[(((rt*D + i)*nkb + kb)*64 + lane)*16 + jj] = digit i of
// psi[slot_src(2 rt + (lane%32 >> 2 & 1), (lane%32 >> 3) * 4 + lane%4)][32 kb + (lane/32)*16 + jj].
// With fold set and the item's fold flag (tile-pair kernel), the last K-block holds A'_i instead: its
// k-slot R2 J + t (R2 = T - 32 (nkb - 1) rows) carries digit i - J of
// psi[row][32 (nkb - 1) + t] for J <= i, 0 otherwise; the reduction kernel
// stores digit J of those target rows at the same k-slot of plane 0.
__global__ __launch_bounds__(256) void k_pack_psi(const DevItem *__restrict__ items,
                                                  const DevDigitItem *__restrict__ ditems,
                                                  const int16_t *__restrict__ slot_src, int nrt, int nkb, int T,
                                                  int nsrc, int fold) {
    const DevItem it = items[blockIdx.y];
    const DevDigitItem dd = ditems[blockIdx.y];
    const int D = dd.D;
    const int n = nrt * nkb * 64 * 16;  // entries per digit plane
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const int jj = e & 15, lane = (e >> 4) & 63, rest = e >> 10;
    const int kb = rest % nkb, rt = rest / nkb;
    const int rho = lane & 31, hh = (rho >> 2) & 1, js = (rho >> 3) * 4 + (rho & 3);
    const int row = slot_src[(2 * rt + hh) * 16 + js];
    const int kslot = (lane >> 5) * 16 + jj;
    const bool folded = fold && dd.fold && kb == nkb - 1;
    const int base = 32 * (nkb - 1), r2 = T - base;
    const int Jf = folded ? kslot / r2 : 0;  // plane whose folded rows this k-slot carries
    const int k = folded ? base + kslot % r2 : 32 * kb + kslot;
    const bool inside = row >= 0 && row < nsrc && k < T && (!folded || Jf < D);
    uint64_t x = inside ? it.psi_out[(size_t)row * T + k] : 0;
    // balanced digits of x = unsigned digits of (x + (Q'-1)/2) mod Q', minus (B-1)/2
    const uint64_t Q = dd.Qp, bias = (Q - 1) / 2, B = (uint64_t)dd.B;
    x += bias;
    if (x >= Q) x -= Q;
    int8_t *out = dd.apack_out + ((size_t)(rt * D) * nkb + kb) * 1024 + (size_t)lane * 16 + jj;
    int8_t dig[16];
    // x < Q' < 2^52 is exact in fp64: the quotient by B from the product with
    // 1 / B is off by at most one, which the remainder's range corrects (a
    // 64-bit integer division costs far more on the GPU)
    const double invB = 1.0 / (double)dd.B;
    for (int i = 0; i < D; i++) {
        uint64_t qd = (uint64_t)((double)x * invB);
        int64_t r = (int64_t)(x - qd * B);
        if (r < 0) {
            qd--;
            r += (int64_t)B;
        } else if (r >= (int64_t)B) {
            qd++;
            r -= (int64_t)B;
        }
        dig[i] = (int8_t)((int)r - dd.halfB);
        x = qd;
    }
    // unfolded: fragment i holds digit i; folded: fragment i holds digit i - Jf
    for (int i = 0; i < D; i++) out[(size_t)i * nkb * 1024] = !folded ? dig[i] : (inside && Jf <= i ? dig[i - Jf] : 0);
}

// The same elimination spread over the whole device, for families whose
// [J | I] is too large for one workgroup to stream once per pivot (quintic
// surfaces: 560 x 1440 words per item).  Per pivot row r, one launch finds
// the pivot of every item (one wave each: the first unused column holding a
// unit mod p, its inverse, the row scaled, the pivot column snapshot), and
// one launch clears that column from every other row of every item (one wave
// per row, skipping the rows already zero there).  The pivots, and so psi,
// are those of the one-workgroup form.  Per-item bookkeeping in `book`:
// used[C] (pivot row + 1 of each column), fcol[R], then {pivot column,
// failure} and the pivot inverse.
constexpr int kGjWaves = 4;

struct GjBook {
    int *used;
    uint64_t *fcol;
    int *state;
    uint64_t *inv;
};

__device__ __forceinline__ static GjBook gj_book(unsigned char *book, int item, int R, int C) {
    unsigned char *b = book + (size_t)item * gj_book_bytes(R, C);
    GjBook g;
    g.fcol = reinterpret_cast<uint64_t *>(b);
    g.inv = g.fcol + R;
    g.used = reinterpret_cast<int *>(g.inv + 1);
    g.state = g.used + C;
    return g;
}

// [J | I] rows and cleared bookkeeping; grid (row blocks, items)
__global__ __launch_bounds__(64 * kGjWaves) void k_gj_init(const DevItem *__restrict__ items, int R, int C,
                                                            const int32_t *__restrict__ jtab, uint64_t *work,
                                                            unsigned char *book) {
    const DevItem it = items[blockIdx.y];
    if (it.q == 0) return;
    const PMod md{it.q, it.mu, it.sbits};
    const int W = C + R, lane = threadIdx.x & 63, r = blockIdx.x * kGjWaves + (threadIdx.x >> 6);
    uint64_t *a = work + (size_t)blockIdx.y * R * W;
    const GjBook g = gj_book(book, blockIdx.y, R, C);
    if (r < R)
        for (int k = lane; k < W; k += 64)
            if (k < C) {
                const int32_t e = jtab[(size_t)r * C + k];
                a[(size_t)r * W + k] = e < 0 ? 0 : md.reduce((u128p)it.fcoef[e >> 8] * (uint32_t)(e & 255));
            } else {
                a[(size_t)r * W + k] = (uint64_t)(k - C == r);
            }
    for (int k = blockIdx.x * 64 * kGjWaves + threadIdx.x; k < C; k += gridDim.x * 64 * kGjWaves) g.used[k] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) g.state[0] = g.state[1] = 0;
}

// pivot of row r of every item: one wave per item
__global__ __launch_bounds__(64) void k_gj_pivot(const DevItem *__restrict__ items, int R, int C, int r,
                                                 uint64_t *work, unsigned char *book) {
    const DevItem it = items[blockIdx.x];
    if (it.q == 0) return;
    const GjBook g = gj_book(book, blockIdx.x, R, C);
    if (g.state[1]) return;  // uniform over the wave
    const PMod md{it.q, it.mu, it.sbits};
    const uint32_t p = (uint32_t)it.p, two32p = (uint32_t)((1ull << 32) % p);
    const int W = C + R, lane = threadIdx.x;
    uint64_t *a = work + (size_t)blockIdx.x * R * W;
    uint64_t *row = a + (size_t)r * W;
    int c = C;
    for (int k0 = 0; k0 < C && c == C; k0 += 64) {
        const int k = k0 + lane;
        const bool ok = k < C && !g.used[k] && mod_small(row[k], p, two32p) != 0;
        const unsigned long long m = __ballot(ok);
        if (m) c = k0 + __ffsll((long long)m) - 1;
    }
    if (c == C) {  // J_S is not surjective mod p
        if (lane == 0) {
            g.state[1] = 1;
            atomicOr(it.flag, 1);
        }
        return;
    }
    uint64_t inv = 0;
    if (lane == 0) inv = inv_mod(md, row[c], p, two32p);
    inv = __shfl(inv, 0);
    for (int r2 = lane; r2 < R; r2 += 64) g.fcol[r2] = r2 == r ? 0 : a[(size_t)r2 * W + c];
    for (int k = lane; k < W; k += 64) row[k] = md.mul(row[k], inv);
    if (lane == 0) {
        g.used[c] = r + 1;
        g.state[0] = c;
    }
}

// column c_r cleared from every other row: grid (row blocks, items), one wave per row
__global__ __launch_bounds__(64 * kGjWaves) void k_gj_update(const DevItem *__restrict__ items, int R, int C, int r,
                                                              uint64_t *work, unsigned char *book) {
    const DevItem it = items[blockIdx.y];
    if (it.q == 0) return;
    const GjBook g = gj_book(book, blockIdx.y, R, C);
    if (g.state[1]) return;
    const int r2 = blockIdx.x * kGjWaves + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r2 >= R) return;
    const uint64_t f = g.fcol[r2];
    if (f == 0) return;  // row r itself, and rows already zero in the pivot column
    const PMod md{it.q, it.mu, it.sbits};
    const int W = C + R;
    uint64_t *a = work + (size_t)blockIdx.y * R * W;
    const uint64_t *row = a + (size_t)r * W;
    uint64_t *o = a + (size_t)r2 * W;
    for (int k = lane; k < W; k += 64) {
        const uint64_t y = row[k];
        if (y == 0) continue;
        const uint64_t t = md.mul(f, y);
        const uint64_t x = o[k];
        o[k] = x >= t ? x - t : x + md.q - t;
    }
}

// psi (C x R): row c = pivot of row r -> right half of row r; grid (column blocks, items)
__global__ __launch_bounds__(64 * kGjWaves) void k_gj_emit(const DevItem *__restrict__ items, int R, int C,
                                                            const uint64_t *work, unsigned char *book) {
    const DevItem it = items[blockIdx.y];
    if (it.q == 0) return;
    const GjBook g = gj_book(book, blockIdx.y, R, C);
    const bool fail = g.state[1] != 0;
    const int cc = blockIdx.x * kGjWaves + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (cc >= C) return;
    const int r1 = g.used[cc];
    const uint64_t *a = work + (size_t)blockIdx.y * R * (C + R);
    for (int j = lane; j < R; j += 64)
        it.psi_out[(size_t)cc * R + j] = (!fail && r1 > 0) ? a[(size_t)(r1 - 1) * (C + R) + C + j] : 0;
}

size_t psi_book_bytes(int R, int C) { return gj_book_bytes(R, C); }

hipError_t launch_psi_multi(const DevItem *items, int nitems, int R, int C, const int32_t *jtab, uint64_t *work,
                            unsigned char *book, hipStream_t stream) {
    if (nitems == 0) return hipSuccess;
    const dim3 rows((R + kGjWaves - 1) / kGjWaves, nitems), block(64 * kGjWaves);
    hipLaunchKernelGGL(k_gj_init, rows, block, 0, stream, items, R, C, jtab, work, book);
    for (int r = 0; r < R; r++) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(nitems), dim3(64), 0, stream, items, R, C, r, work, book);
        hipLaunchKernelGGL(k_gj_update, rows, block, 0, stream, items, R, C, r, work, book);
    }
    hipLaunchKernelGGL(k_gj_emit, dim3((C + kGjWaves - 1) / kGjWaves, nitems), block, 0, stream, items, R, C,
                       (const uint64_t *)work, book);
    return hipGetLastError();
}

hipError_t launch_psi(const DevItem *items, int nitems, int R, int C, const int32_t *jtab, hipStream_t stream) {
    if (nitems == 0) return hipSuccess;
    const size_t lds = psi_lds_bytes(R, C);
    hipError_t e = hipFuncSetAttribute((const void *)k_psi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_psi, dim3(nitems), dim3(kPsiThreads), lds, stream, items, R, C, jtab);
    return hipGetLastError();
}

hipError_t launch_psi_global(const DevItem *items, int nitems, int R, int C, const int32_t *jtab, uint64_t *work,
                             hipStream_t stream) {
    if (nitems == 0) return hipSuccess;
    const size_t lds = psi_small_lds_bytes(R, C);
    hipLaunchKernelGGL(k_psi_global, dim3(nitems), dim3(kPsiThreads), lds, stream, items, R, C, jtab, work);
    return hipGetLastError();
}

hipError_t launch_pack_psi(const DevItem *items, const DevDigitItem *ditems, int nitems, const int16_t *slot_src,
                           int nrt, int nkb, int T, int nsrc, int fold, hipStream_t stream) {
    if (nitems == 0) return hipSuccess;
    const int n = nrt * nkb * 64 * 16;
    hipLaunchKernelGGL(k_pack_psi, dim3((n + 255) / 256, nitems), dim3(256), 0, stream, items, ditems, slot_src, nrt,
                       nkb, T, nsrc, fold);
    return hipGetLastError();
}

}  // namespace crf
