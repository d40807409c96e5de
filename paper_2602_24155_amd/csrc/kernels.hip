// HIP kernels (gfx950) for the controlled-reduction hot loop.
//
// k_reduce_chains: every Frobenius start term (Proposition 2.1) is one chain
//   x^{u0} x^gamma / (x^S f^P)  ->  pole n,
// reduced one pole order per step with R_{u,v} (Proposition 3.3).  With psi a
// right inverse of J_S, the explicit formula of Section 3.1 gives
//   R_{u,v}[r, g] = sum_i (u_i + r_i + [i not in S]) psi_i[r - 1_S + [i in S] e_i, v + g - 1_S],
// so one step is  t = psi[:, cols(v)] w  followed by a weighted gather
//   w'[r] = sum_i (u_i + r_i + [i not in S]) t[src(r, i)]      (mod p^M),
// u the exponent after the step.  v is chosen by Algorithm 3 at the start of
// each chunk and kept for the largest k allowed (depth-first policy, Section
// 4.2); inside a chunk the matrices M(y) = R_{x + y v, v} are applied from
// y = k-1 down to 0 as in Algorithm 2, with M(y) never materialised.
//
// A chain is one vector of a reduction plan: it may start from a stored
// residue vector instead of e_gamma, stop at a combine point (pole pend > n)
// and leave its result in a store row, and may have one direction forced for
// its whole range (the learned policy).
//
// k_combine: store rows built between phases (like terms combined, Section 3.4).
// k_assemble_h / k_assemble_y: H = sum coef (x) h over the vectors that reach
// pole n, and Y = rho H (Section 3.3 step (2)).
#include <hip/hip_runtime.h>

#include "device_layout.hpp"

namespace crf {

typedef unsigned __int128 u128;
typedef uint64_t u64;

struct DMod {
    u64 q, mu;
    int sbits;
    __device__ __forceinline__ u64 reduce(u128 x) const {
        u64 x1 = (u64)(x >> (sbits - 1));
        u128 prod = (u128)x1 * mu;
        u64 qh = (u64)(prod >> (sbits + 9));
        u64 r = (u64)x - qh * q;
        r = r >= q ? r - q : r;
        r = r >= q ? r - q : r;
        return r;
    }
};

// Algorithm 3 (greedy v) for the current exponent U; returns the direction
// index and the chunk length k = largest with U - k v >= 0 (capped by the
// remaining pole orders).  Validity (i in S, U_i != 0 => v_i != 0) holds by
// construction when d >= |S|.
__device__ static void choose_chunk(const DevFamily &fam, const int *U, int poles_left, int *v, int &dir, int &k) {
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

constexpr int kThreads = 256;

// Dynamic LDS layout per workgroup (ct chains):
//   w  : ct x s    u64
//   t  : ct x nsrc u64
//   U, v : ct x 8 int ; dir, kleft, pole : ct int
__global__ __launch_bounds__(kThreads) void k_reduce_chains(DevFamily fam, const DevItem *__restrict__ items,
                                                            const DevTile *__restrict__ tiles,
                                                            const int16_t *__restrict__ cu,
                                                            const int32_t *__restrict__ cg,
                                                            const int32_t *__restrict__ cpole,
                                                            const DevVec *__restrict__ vx,
                                                            u64 *__restrict__ store,
                                                            u64 *__restrict__ hbuf, int ct,
                                                            int *__restrict__ err) {
    extern __shared__ __align__(16) unsigned char lds[];
    const DevTile tile = tiles[blockIdx.x];
    const DevItem it = items[tile.item];
    const DMod md{it.q, it.mu, it.sbits};
    const int s = fam.s, nsrc = fam.nsrc, T = fam.T, nv = fam.nv;
    u64 *w = reinterpret_cast<u64 *>(lds);
    u64 *t = w + (size_t)ct * s;
    int *U = reinterpret_cast<int *>(t + (size_t)ct * nsrc);
    int *V = U + ct * 8;
    int *dir = V + ct * 8;
    int *kleft = dir + ct;
    int *pole = kleft + ct;
    int *pend = pole + ct;
    const int tid = threadIdx.x;
    const int nch = tile.count;

    for (int idx = tid; idx < ct * s; idx += kThreads) w[idx] = 0;
    __syncthreads();
    if (tid < nch) {
        const int g = tile.chain0 + tid;
        const DevVec x = vx[g];
        for (int i = 0; i < nv; i++) U[tid * 8 + i] = cu[(size_t)g * nv + i];
        pole[tid] = cpole[g];
        pend[tid] = x.pend;
        kleft[tid] = 0;
        if (x.dir >= 0) {  // one forced direction for the whole range
            for (int i = 0; i < nv; i++) V[tid * 8 + i] = fam.dirs[x.dir * nv + i];
            dir[tid] = x.dir;
            kleft[tid] = pole[tid] - x.pend;
        }
        if (x.in < 0) w[tid * s + cg[g]] = 1;
    }
    for (int idx = tid; idx < nch * s; idx += kThreads) {
        const int c = idx / s, r = idx - c * s;
        const int in = vx[tile.chain0 + c].in;
        if (in >= 0) w[idx] = store[(size_t)in * s + r];
    }
    __syncthreads();

    for (int step = 0; step < tile.steps; step++) {
        if (tid < nch && pole[tid] > pend[tid] && kleft[tid] == 0) {
            int d0, k0;
            choose_chunk(fam, &U[tid * 8], pole[tid] - pend[tid], &V[tid * 8], d0, k0);
            if (d0 < 0 || k0 < 1) {  // no valid direction: cannot happen for d >= |S|
                atomicOr(err, 1);
                d0 = 0;
                k0 = 1 << 30;
                pole[tid] = pend[tid];
            }
            dir[tid] = d0;
            kleft[tid] = k0;
        }
        __syncthreads();
        // t = psi[:, cols(v)] w
        for (int idx = tid; idx < nch * nsrc; idx += kThreads) {
            const int c = idx / nsrc, mu = idx - c * nsrc;
            if (pole[c] <= pend[c]) continue;
            const int16_t *cm = fam.colmap + (size_t)dir[c] * s;
            const u64 *prow = it.psi + (size_t)mu * T;
            const u64 *wc = w + (size_t)c * s;
            u128 acc = 0;
            for (int k = 0; k < s; k++) {
                const int col = cm[k];
                const u64 x = wc[k];
                if (x) {
                    if (col >= 0) acc += (u128)prow[col] * x;
                    else atomicOr(err, 2);  // x^v g / x^S not a polynomial: invariant broken
                }
                if ((k & 255) == 255) acc = md.reduce(acc);
            }
            t[(size_t)c * nsrc + mu] = md.reduce(acc);
        }
        __syncthreads();
        // w'[r] = sum_i (u_i + r_i + [i not in S]) t[src(r, i)],  u = U - v
        for (int idx = tid; idx < nch * s; idx += kThreads) {
            const int c = idx / s, r = idx - c * s;
            if (pole[c] <= pend[c]) continue;
            u128 acc = 0;
            for (int i = 0; i < nv; i++) {
                const int src = fam.gsrc[r * nv + i];
                if (src < 0) continue;
                const u64 wt = (u64)(U[c * 8 + i] - V[c * 8 + i] + fam.gw[r * nv + i]);
                acc += (u128)wt * t[(size_t)c * nsrc + src];
            }
            w[(size_t)c * s + r] = md.reduce(acc);
        }
        __syncthreads();
        if (tid < nch && pole[tid] > pend[tid]) {
            for (int i = 0; i < nv; i++) U[tid * 8 + i] -= V[tid * 8 + i];
            pole[tid]--;
            kleft[tid]--;
        }
        __syncthreads();
    }
    // combine point: the vector goes to its store row
    for (int idx = tid; idx < nch * s; idx += kThreads) {
        const int c = idx / s, r = idx - c * s;
        const int out = vx[tile.chain0 + c].out;
        if (out >= 0) store[(size_t)out * s + r] = w[idx];
    }
    // pole n: numerator x^U g / x^S written into fin space
    for (int c = 0; c < nch; c++) {
        if (vx[tile.chain0 + c].out >= 0) continue;
        u64 *h = hbuf + (size_t)(tile.chain0 + c) * fam.F;
        for (int f = tid; f < fam.F; f += kThreads) h[f] = 0;
    }
    __syncthreads();
    for (int idx = tid; idx < nch * s; idx += kThreads) {
        const int c = idx / s, k = idx - c * s;
        if (vx[tile.chain0 + c].out >= 0) continue;
        int Ui = -1;
        for (int a = 0; a < fam.nfinU && Ui < 0; a++) {
            bool eq = true;
            for (int i = 0; i < nv; i++) eq = eq && (fam.finU[a * nv + i] == U[c * 8 + i]);
            if (eq) Ui = a;
        }
        const u64 x = w[(size_t)c * s + k];
        if (!x) continue;
        const int f = Ui < 0 ? -1 : fam.finmap[(size_t)Ui * s + k];
        if (f >= 0) hbuf[(size_t)(tile.chain0 + c) * fam.F + f] = x;
        else atomicOr(err, 4);
    }
}

// Store rows built between two phases: row = sum_j alpha_j src_j (mod q).
__global__ __launch_bounds__(64) void k_combine(const DevItem *__restrict__ items, const DevComb *__restrict__ comb,
                                                const int32_t *__restrict__ msrc, const u64 *__restrict__ malpha,
                                                u64 *__restrict__ store, int s) {
    const DevComb cb = comb[blockIdx.x];
    const DevItem it = items[cb.item];
    const DMod md{it.q, it.mu, it.sbits};
    for (int r = threadIdx.x; r < s; r += 64) {
        u128 acc = 0;
        for (int j = cb.m0; j < cb.m1; j++) {
            const int src = msrc[j];
            const u64 x = src >= 0 ? store[(size_t)src * s + r] : (u64)(r == -src - 1);
            acc += (u128)malpha[j] * x;
            if (((j - cb.m0) & 127) == 127) acc = md.reduce(acc);
        }
        store[(size_t)cb.row * s + r] = md.reduce(acc);
    }
}

// H = sum_k h_k (x) coef_k over the vectors that reach pole n: one workgroup
// per (item, row f of H).  Thread t takes column c = t mod b and every
// (kThreads / b)-th vector of its slice; the slices are summed in LDS.
__global__ __launch_bounds__(kThreads) void k_assemble_h(DevFamily fam, const DevItem *__restrict__ items,
                                                         const u64 *__restrict__ hbuf) {
    __shared__ u64 part[kThreads];
    const DevItem it = items[blockIdx.x];
    const int f = blockIdx.y;
    const DMod md{it.q, it.mu, it.sbits};
    const int F = fam.F, b = it.b, t = threadIdx.x;
    const int nsl = kThreads / b;  // b <= kThreads
    const int c = t % b, sl = t / b;
    u64 r = 0;
    if (sl < nsl) {
        u128 acc = 0;
        int cnt = 0;
        for (int k = sl; k < it.nfin; k += nsl) {
            const u64 h = hbuf[(size_t)it.fvec[k] * F + f];
            if (h) acc += (u128)h * it.coef[(size_t)it.frow[k] * b + c];
            if (++cnt == 128) {
                acc = md.reduce(acc);
                cnt = 0;
            }
        }
        r = md.reduce(acc);
    }
    part[t] = r;
    __syncthreads();
    if (t < b) {
        u128 acc = 0;
        for (int j = 0; j < nsl; j++) acc += part[j * b + t];
        it.H[(size_t)f * b + t] = md.reduce(acc);
    }
}

// Y = rho H, one workgroup per item.
__global__ __launch_bounds__(kThreads) void k_assemble_y(DevFamily fam, const DevItem *__restrict__ items) {
    const DevItem it = items[blockIdx.x];
    const DMod md{it.q, it.mu, it.sbits};
    const int F = fam.F, b = it.b;
    for (int idx = threadIdx.x; idx < b * b; idx += kThreads) {
        const int i = idx / b, c = idx - i * b;
        u128 acc = 0;
        for (int f = 0; f < F; f++) {
            acc += (u128)it.rho[(size_t)i * F + f] * it.H[(size_t)f * b + c];
            if ((f & 127) == 127) acc = md.reduce(acc);
        }
        it.Y[idx] = md.reduce(acc);
    }
}

size_t reduce_lds_bytes(const DevFamily &fam, int ct) {
    return (size_t)ct * (fam.s + fam.nsrc) * 8 + (size_t)ct * (8 + 8 + 4) * 4;
}

hipError_t launch_reduce(const DevFamily &fam, const DevItem *items, const DevTile *tiles, int ntiles,
                         const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx, u64 *store,
                         u64 *hbuf, int ct, int *err, hipStream_t stream) {
    if (ntiles == 0) return hipSuccess;
    size_t lds = reduce_lds_bytes(fam, ct);
    hipLaunchKernelGGL(k_reduce_chains, dim3(ntiles), dim3(kThreads), lds, stream, fam, items, tiles, cu, cg, cpole,
                       vx, store, hbuf, ct, err);
    return hipGetLastError();
}

hipError_t launch_combine(const DevItem *items, const DevComb *comb, int ncomb, const int32_t *msrc,
                          const u64 *malpha, u64 *store, int s, hipStream_t stream) {
    if (ncomb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine, dim3(ncomb), dim3(64), 0, stream, items, comb, msrc, malpha, store, s);
    return hipGetLastError();
}

hipError_t launch_assemble(const DevFamily &fam, const DevItem *items, int nitems, const u64 *hbuf,
                           hipStream_t stream) {
    if (nitems == 0) return hipSuccess;
    if (fam.F > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_assemble_h, dim3(nitems, fam.F), dim3(kThreads), 0, stream, fam, items, hbuf);
    hipLaunchKernelGGL(k_assemble_y, dim3(nitems), dim3(kThreads), 0, stream, fam, items);
    return hipGetLastError();
}

}  // namespace crf
