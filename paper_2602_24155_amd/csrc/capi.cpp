// C-ABI entry points of libcrfrob.so (declared in include/crfrob.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "device_layout.hpp"
#include "devmem.hpp"
#include "host.hpp"
#include "mlp.hpp"
#include "plan.hpp"

namespace crf {
size_t reduce_lds_bytes(const DevFamily &fam, int ct);
hipError_t launch_reduce(const DevFamily &fam, const DevItem *items, const DevTile *tiles, int ntiles,
                         const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                         uint64_t *store, uint64_t *hbuf, int ct, int *err, hipStream_t stream);
hipError_t launch_combine(const DevItem *items, const DevComb *comb, int ncomb, const int32_t *msrc,
                          const uint64_t *malpha, uint64_t *store, int s, hipStream_t stream);
hipError_t launch_assemble(const DevFamily &fam, const DevItem *items, int nitems, const uint64_t *hbuf,
                           hipStream_t stream);
bool mfma_shape(const DevFamily &fam, int &nrt, int &nkb);
bool mfma4_shape(const DevFamily &fam, int &nrt, int &nkb);
hipError_t launch_reduce_mfma(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, uint64_t *hbuf, int *err,
                              int D, hipStream_t stream);
bool mfma_supports_digits(int D);
hipError_t launch_reduce_mfma4(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                               const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                               uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int D, bool z32,
                               int pgrid, int *queue, hipStream_t stream);
hipError_t launch_zero_ints(int *p, int n, hipStream_t stream);
bool mfma5_supports(const DevFamily &fam, int D);
hipError_t launch_reduce_mfma5(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int npairs,
                               const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                               uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int D, bool z32,
                               int pgrid, int *queue, hipStream_t stream);
size_t psi_lds_bytes(int R, int C);
hipError_t launch_psi(const DevItem *items, int nitems, int R, int C, const int32_t *jtab, hipStream_t stream);
hipError_t launch_psi_multi(const DevItem *items, int nitems, int R, int C, const int32_t *jtab, uint64_t *work,
                            unsigned char *book, hipStream_t stream);
size_t psi_book_bytes(int R, int C);
hipError_t launch_psi_global(const DevItem *items, int nitems, int R, int C, const int32_t *jtab, uint64_t *work,
                             hipStream_t stream);
hipError_t launch_pack_psi(const DevItem *items, const DevDigitItem *ditems, int nitems, const int16_t *slot_src,
                           int nrt, int nkb, int T, int nsrc, int fold, hipStream_t stream);
bool mfma4_supports(const DevFamily &fam, int D);
bool quad_shape(const DevFamily &fam, int &nrt, int &nrtf, int &nkb);
bool quad_supports_digits(int D);
hipError_t launch_reduce_quad(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                              uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int pgrid, int *queue,
                              hipStream_t stream);
bool wide_shape(const DevFamily &fam, int &nrt, int &nrtq, int &nkb);
bool wide_supports_digits(int D);
size_t wide_scratch_bytes(int D, int grid);
int wide_grid(int ntiles, int pgrid);
hipError_t launch_reduce_wide(const DevFamily &fam, const DevDigitItem *items, const DevTile *tiles, int ntiles,
                              const int16_t *cu, const int32_t *cg, const int32_t *cpole, const DevVec *vx,
                              uint64_t *store, uint64_t *hbuf, const uint32_t *slots, int *err, int D, int grid,
                              int8_t *xscratch, int *queue, hipStream_t stream);
}  // namespace crf

using namespace crf;

namespace {

thread_local std::string g_err;

}  // namespace

namespace crf {
void set_last_error(const std::string &msg) { g_err = msg; }
}  // namespace crf

namespace {

cr_status fail(cr_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

// ------------------------------------------------------------ device memory
// One grow-only device buffer and one pinned host staging buffer, reused by
// every call (calls are serialised by g_mutex).  A fixed arena (the
// allocation-free entry point) is a slice of the static device workspace
// with pageable host staging: it never allocates device or pinned memory and
// fails when a request exceeds its slice.
struct Arena {
    void *dev = nullptr;
    size_t dev_cap = 0;
    DevBlock block;  // the device buffer of a growing arena
    void *host = nullptr;
    size_t host_cap = 0;
    bool fixed = false;
    std::vector<unsigned char> host_heap;  // host staging of a fixed arena
    void bind(void *slice, size_t bytes) {
        fixed = true;
        dev = slice;
        dev_cap = bytes;
    }
    bool ensure(size_t dbytes, size_t hbytes) {
        if (fixed) {
            if (dbytes > dev_cap) return false;
            if (hbytes > host_heap.size()) host_heap.resize(hbytes);
            host = host_heap.data();
            host_cap = host_heap.size();
            return true;
        }
        if (dbytes > dev_cap) {
            const size_t cap = std::max(dbytes, dev_cap + dev_cap / 2);
            dev_free(block);
            dev = nullptr;
            dev_cap = 0;
            if (!dev_alloc(block, cap)) return false;
            dev = block.ptr;
            dev_cap = cap;
        }
        if (hbytes > host_cap) {
            const size_t cap = std::max(hbytes, host_cap + host_cap / 2);
            if (host) (void)hipHostFree(host);
            host = nullptr;
            host_cap = 0;
            if (hipHostMalloc(&host, cap, hipHostMallocDefault) != hipSuccess) return false;
            host_cap = cap;
        }
        return true;
    }
    void release() {
        if (fixed) return;
        dev_free(block);
        if (host) (void)hipHostFree(host);
        dev = host = nullptr;
        dev_cap = host_cap = 0;
    }
};

struct FamilyEntry {
    Family fam;
    std::vector<unsigned char> tables;  // packed device tables (host copy)
    size_t off_colmap, off_gsrc, off_gw, off_finmap, off_dirs, off_finU, off_slots, off_slot_src, off_qslots, off_qslot_src;
    BinLayout bl;  // source-row placement for the register-gather MFMA kernel
    bool bl_ok = false;
    BinLayout ql;  // row placement of the quad kernel (or of the streaming kernel)
    bool ql_ok = false;
};

std::mutex g_mutex;
constexpr int kArenas = 2;
Arena g_arenas[kArenas];  // sub-batch k of a call uses arena k mod kArenas
Arena g_psi_arena;         // psi of every hypersurface of a call (device psi)
std::map<std::string, hipGraphExec_t> g_graphs;  // captured reduction launches by launch signature
hipStream_t g_capture = nullptr;                 // private stream used for graph capture
hipStream_t g_aux = nullptr;                     // upload and psi of the next sub-batch

void clear_graphs() {
    for (auto &g : g_graphs) (void)hipGraphExecDestroy(g.second);
    g_graphs.clear();
}
std::map<std::tuple<int, int, uint32_t>, std::unique_ptr<FamilyEntry>> g_families;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

FamilyEntry *get_family(const cr_family *fam, std::string &err) {
    auto key = std::make_tuple(fam->nvars, fam->degree, fam->s_mask);
    auto it = g_families.find(key);
    if (it != g_families.end()) return it->second.get();
    auto e = std::make_unique<FamilyEntry>();
    if (!e->fam.init(fam->nvars, fam->degree, fam->s_mask, err)) return nullptr;
    const Family &F = e->fam;
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        e->tables.resize(off);
        std::memcpy(e->tables.data() + at, src, bytes);
        return at;
    };
    e->off_colmap = put(F.colmap.data(), F.colmap.size() * 2);
    e->off_gsrc = put(F.gsrc.data(), F.gsrc.size() * 2);
    e->off_gw = put(F.gw.data(), F.gw.size() * 2);
    e->off_finmap = put(F.finmap.data(), F.finmap.size() * 2);
    e->off_dirs = put(F.dirs.exps.data(), F.dirs.exps.size());
    e->off_finU = put(F.finU.exps.data(), std::max<size_t>(F.finU.exps.size(), 1));
    {
        DevFamily shape{};
        shape.nsrc = F.nsrc;
        shape.T = F.tgt.count;
        shape.s = F.g.count;
        shape.ndir = F.dirs.count;
        shape.nv = F.nv;
        shape.smask = F.smask;
        shape.nfinU = F.finU.count;
        int nrt = 0, nkb = 0;
        e->bl_ok = mfma4_shape(shape, nrt, nkb) && bin_layout(F, nrt, e->bl);
        if (!e->bl_ok) e->bl.slot.assign(16, 0);
        e->off_slots = put(e->bl.slot.data(), e->bl.slot.size() * 4);
        std::vector<int16_t> ss(e->bl.slot_src.begin(), e->bl.slot_src.end());
        if (ss.empty()) ss.assign(16, -1);
        e->off_slot_src = put(ss.data(), ss.size() * 2);
        int qrt = 0, qrtf = 0, qkb = 0;
        // the quad placement (quartic K3 surfaces; quintic surfaces in the streaming
        // kernel) or the quint placement (cubic threefolds)
        if (quad_shape(shape, qrt, qrtf, qkb))
            e->ql_ok = quad_layout(F, qrt, qrtf, e->ql);
        else
            e->ql_ok = wide_shape(shape, qrt, qrtf, qkb) &&
                       (F.nv == 4 ? quad_layout(F, qrt, qrtf, e->ql) : wide_layout(F, qrt, qrtf, e->ql));
        if (!e->ql_ok) e->ql.slot.assign(16, 0);
        e->off_qslots = put(e->ql.slot.data(), e->ql.slot.size() * 4);
        std::vector<int16_t> qs(e->ql.slot_src.begin(), e->ql.slot_src.end());
        if (qs.empty()) qs.assign(16, -1);
        e->off_qslot_src = put(qs.data(), qs.size() * 2);
    }
    auto *raw = e.get();
    g_families.emplace(key, std::move(e));
    return raw;
}

// Persistent worker threads for the per-item host work (at most 16 threads in
// all, the caller included).  A call from inside a task runs serially.
class Pool {
  public:
    static Pool &get() {
        static Pool p;
        return p;
    }
    int width() const { return (int)workers_.size() + 1; }
    void run(int count, const std::function<void(int)> &fn) {
        if (count <= 0) return;
        if (in_task || workers_.empty() || count == 1) {
            for (int i = 0; i < count; i++) fn(i);
            return;
        }
        std::unique_lock<std::mutex> lk(m_);
        job_ = &fn;
        count_ = count;
        next_ = 0;
        busy_ = (int)workers_.size();
        gen_++;
        cv_.notify_all();
        lk.unlock();
        drain();
        lk.lock();
        done_.wait(lk, [&] { return busy_ == 0; });
        job_ = nullptr;
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }

  private:
    Pool() {
        int hw = (int)std::thread::hardware_concurrency();
        const int n = std::max(0, std::min(hw > 0 ? hw : 1, 16) - 1);
        for (int t = 0; t < n; t++) workers_.emplace_back([this] { loop(); });
    }
    void drain() {
        in_task = true;
        for (int i = next_++; i < count_; i = next_++) (*job_)(i);
        in_task = false;
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            std::unique_lock<std::mutex> lk(m_);
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (stop_) return;
            lk.unlock();
            drain();
            lk.lock();
            if (--busy_ == 0) done_.notify_all();
        }
    }
    static thread_local bool in_task;
    std::vector<std::thread> workers_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *job_ = nullptr;
    std::atomic<int> next_{0};
    int count_ = 0, busy_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};
thread_local bool Pool::in_task = false;

// Frees what a finished call leaves behind (the host state of its items and
// plans: thousands of heap blocks for a batch of hundreds of hypersurfaces)
// on a thread of its own, so that the call returns without waiting for the
// frees (about half a millisecond per call for 256 plane quintics).
class Reaper {
  public:
    static Reaper &get() {
        static Reaper r;
        return r;
    }
    void post(std::function<void()> job) {
        {
            std::lock_guard<std::mutex> lk(m_);
            q_.push_back(std::move(job));
        }
        cv_.notify_one();
    }
    ~Reaper() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_one();
        th_.join();
    }

  private:
    Reaper() : th_([this] { loop(); }) {}
    void loop() {
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
            while (!q_.empty()) {
                std::function<void()> job = std::move(q_.front());
                q_.pop_front();
                lk.unlock();
                job();
                job = nullptr;
                lk.lock();
            }
            if (stop_) return;
        }
    }
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<std::function<void()>> q_;
    bool stop_ = false;
    std::thread th_;  // last: starts after the members it uses exist
};

template <class Fn>
void parallel_for(int count, Fn fn) {
    const std::function<void(int)> f = fn;
    Pool::get().run(count, f);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

long long hodge_size(int nv, int d, int m) {
    const int n = nv - 1, k = d * m - n - 1;
    long long h = 0;
    for (int j = 0; j < nv; j++) {
        int kk = k - j * (d - 1);
        if (kk < 0) break;
        h += ((j & 1) ? -1 : 1) * binom(nv, j) * count_monomials(nv, kk);
    }
    return h;
}

bool check_family(const cr_family *fam, std::string &err) {
    if (!fam) {
        err = "null family";
        return false;
    }
    if (fam->nvars < 3 || fam->nvars > kMaxVars || fam->degree < 2 || fam->degree > 12) {
        err = "unsupported nvars/degree";
        return false;
    }
    if (fam->engine < 0 || fam->engine > 5) {
        err = "unknown engine";
        return false;
    }
    if (fam->policy < CR_POLICY_DEPTH_FIRST || fam->policy > CR_POLICY_LEARNED) {
        err = "unknown policy";
        return false;
    }
    if (fam->launch < 0 || fam->launch > 2) {
        err = "unknown launch mode";
        return false;
    }
    if (fam->grid < 0 || fam->grid > 4) {
        err = "persistent grid must be 0..4 workgroups per CU";
        return false;
    }
    if (fam->policy != CR_POLICY_DEPTH_FIRST && fam->engine == 2) {
        err = "engine 2 (LDS-gather MFMA kernel) runs the depth-first policy only";
        return false;
    }
    return true;
}

// CR_POLICY_LEARNED: the p-chunk phases of every item advance together; per
// phase the candidates of all items are scored in one network evaluation on
// the GPU and every term takes its lowest-scoring candidate.  Each finished
// plan is judged against the depth-first and p-chunk plans (plan_cost) and
// the cheapest is kept.
bool plan_learned(const Family &F, std::vector<ItemSetup> &items, std::vector<cr_status> &st,
                  std::vector<std::string> &errs, std::vector<ItemPlan> &plans, cr_mlp *mlp, hipStream_t stream,
                  int &fallbacks, std::string &err) {
    const int count = (int)items.size();
    std::vector<PChunkPlanner> pl(count);
    std::vector<char> on(count, 0);
    for (int i = 0; i < count; i++) {
        if (st[i] != CR_OK) continue;
        if (!pl[i].init(F, items[i], CR_POLICY_LEARNED, errs[i])) {
            st[i] = CR_EINVAL;
            continue;
        }
        on[i] = 1;
    }
    std::vector<std::vector<CandRow>> rows(count);
    std::vector<char> active(count, 0);
    for (;;) {
        parallel_for(count, [&](int i) {
            active[i] = 0;
            rows[i].clear();
            if (!on[i] || st[i] != CR_OK) return;
            if (!pl[i].begin_phase()) return;
            active[i] = 1;
            pl[i].candidates(rows[i]);
        });
        std::vector<size_t> r0(count + 1, 0);
        bool any = false;
        for (int i = 0; i < count; i++) {
            r0[i + 1] = r0[i] + rows[i].size();
            any = any || active[i];
        }
        if (!any) break;
        const size_t R = r0[count];
        if (R >= (size_t)INT32_MAX) {
            err = "too many candidate rows";
            return false;
        }
        std::vector<float> X(R * kMlpIn), Y(R);
        for (int i = 0; i < count; i++)
            for (size_t k = 0; k < rows[i].size(); k++)
                std::memcpy(&X[(r0[i] + k) * kMlpIn], rows[i][k].x, sizeof(float) * kMlpIn);
        if (!mlp_score(mlp, X.data(), (int)R, Y.data(), stream, err)) return false;
        parallel_for(count, [&](int i) {
            if (!active[i]) return;
            std::vector<int32_t> dir(pl[i].act.size(), -1);
            std::vector<float> best(pl[i].act.size(), 0.f);
            for (size_t k = 0; k < rows[i].size(); k++) {
                const CandRow &r = rows[i][k];
                const float y = Y[r0[i] + k];
                if (dir[r.term] < 0 || y < best[r.term]) {  // rows come in increasing direction order
                    dir[r.term] = r.dir;
                    best[r.term] = y;
                }
            }
            if (!pl[i].end_phase(dir, errs[i])) {
                st[i] = CR_ESELFCHECK;
                on[i] = 0;
            }
        });
    }
    std::atomic<int> fb{0};
    parallel_for(count, [&](int i) {
        if (!on[i] || st[i] != CR_OK) return;
        plans[i] = std::move(pl[i].plan);
        for (int alt : {CR_POLICY_P_CHUNK, CR_POLICY_DEPTH_FIRST}) {
            ItemPlan other;
            std::string e2;
            if (plan_item(F, items[i], alt, other, e2) && plan_cost(other) < plan_cost(plans[i])) {
                if (plans[i].policy == CR_POLICY_LEARNED) fb++;
                plans[i] = std::move(other);
            }
        }
    });
    fallbacks = fb.load();
    return true;
}

// ------------------------------------------------------------------ batch execution
struct Outputs {
    uint64_t *frob, *frob_scaled;
    int32_t *col_pole, *col_prec;
    int64_t *lpoly;
};

// Per-call data shared by the sub-batches.
struct BatchCtx {
    const cr_family *fam = nullptr;
    FamilyEntry *fe = nullptr;
    const Family *F = nullptr;
    DevFamily df{};
    int nco = 0, sdim = 0, b = 0, nrt = 0, nkb = 0, policy = 0;
    bool want_mfma = false, use_bins = false;
    bool quad = false;        // four-variable int8-digit MFMA kernel (k_reduce_quad)
    bool wide = false;        // streaming int8-digit MFMA kernel (k_reduce_wide: threefolds, quintic surfaces)
    bool psi_global = false;  // device psi with [J | I] in global memory (k_psi_global)
    bool psi_multi = false;   // the same elimination spread over the device (k_gj_*)
    bool device_psi = false;  // psi computed by k_psi (its [J | I] fits in LDS)
    bool pairs = false;       // two interleaved tiles per workgroup (k_reduce_mfma5)
    hipStream_t stream = nullptr;
    // device psi: one k_psi launch for every item of the call, at its start
    uint64_t *psi_dev = nullptr;         // count x (nsrc x T), caller's item order
    size_t psi_bytes = 0;                // device bytes of the call's psi region
    const int32_t *psi_flags = nullptr;  // host copy of k_psi's per-item flags (after psi_done)
    hipEvent_t psi_t0 = nullptr, psi_done = nullptr;
    const int32_t *primes = nullptr;
    const uint32_t *coeffs = nullptr;
    Outputs out{};
    // the allocation-free entry point binds these to slices of the static
    // workspace and runs everything on the caller's stream
    bool noalloc = false;
    Arena *arenas[kArenas] = {&g_arenas[0], &g_arenas[1]};
    Arena *psi_arena = &g_psi_arena;
    // stream of the uploads and psi work that overlap the reductions
    hipError_t aux(hipStream_t &out_stream) {
        if (noalloc) {
            out_stream = stream;
            return hipSuccess;
        }
        hipError_t e = hipSuccess;
        if (!g_aux) e = hipStreamCreateWithFlags(&g_aux, hipStreamNonBlocking);
        out_stream = g_aux;
        return e;
    }
    bool init(const cr_family *f, const int32_t *pr, const uint32_t *co, hipStream_t s, std::string &err) {
        fam = f;
        primes = pr;
        coeffs = co;
        stream = s;
        fe = get_family(f, err);
        if (!fe) return false;
        F = &fe->fam;
        int32_t nco_, s_dim, b_;
        cr_query_dims(f->nvars, f->degree, &nco_, &s_dim, &b_);
        nco = nco_;
        b = b_;
        if (b > 256) {
            err = "basis larger than 256 columns";
            return false;
        }
        sdim = F->g.count;
        df.nv = F->nv;
        df.n = F->n;
        df.d = F->d;
        df.smask = F->smask;
        df.s = F->g.count;
        df.T = F->tgt.count;
        df.nsrc = F->nsrc;
        df.F = F->fin.count;
        df.ndir = F->dirs.count;
        df.nfinU = F->finU.count;
        policy = f->policy;
        // engine 0: register-gather kernel (source rows placed by the bin layout); 2: LDS-gather kernel
        use_bins = (f->engine == 0 || f->engine == 3) && fe->bl_ok;
        pairs = f->engine == 0;  // engine 3: the single-tile kernel
        int qrtf = 0;
        quad = (f->engine == 0 || f->engine == 4) && fe->ql_ok && quad_shape(df, nrt, qrtf, nkb);
        wide = !quad && (f->engine == 0 || f->engine == 5) && fe->ql_ok && wide_shape(df, nrt, qrtf, nkb);
        want_mfma = quad || wide || (f->engine == 0 || f->engine == 2 || f->engine == 3) &&
                    (use_bins ? mfma4_shape(df, nrt, nkb) : mfma_shape(df, nrt, nkb));
        // the LDS-gather kernel (engine 2) keeps host psi and host packing
        device_psi = f->engine != 2 && psi_lds_bytes(F->tgt.count, F->nsrc) <= 150 * 1024;
        if (quad) {  // device psi ([J | I] in global memory when it outgrows the LDS), digits in the quad placement
            use_bins = pairs = false;
            device_psi = true;
            psi_global = psi_lds_bytes(F->tgt.count, F->nsrc) > 150 * 1024;
        }
        if (wide) {
            // device psi by the device-wide elimination ([J | I] of 6.5 MB per quintic
            // surface, 22 MB per cubic threefold), digits packed on the device in the quad
            // or quint placement
            use_bins = pairs = false;
            device_psi = psi_multi = true;
        }
        // without an MFMA kernel the 64-bit VALU kernel reads psi[:, cols(v)] from memory
        // for every step of every vector, two vectors per workgroup when psi is large;
        // beyond 2^20 entries (cubic threefolds: 1815 x 1001, 716k column steps over F_7,
        // some petabytes of psi reads, minutes per hypersurface; cubic fourfolds: 80 million
        // entries) such families are refused
        if (!want_mfma && (size_t)F->nsrc * F->tgt.count > ((size_t)1 << 20)) {
            err = "no device path for this family: psi has " + std::to_string((size_t)F->nsrc * F->tgt.count) +
                  " entries (the 64-bit kernel handles up to 2^20)";
            return false;
        }
        return true;
    }
};

struct SubBatch {
    std::vector<int> idx;  // caller item indices
    int arena = 0;
    std::vector<ItemSetup> items;
    std::vector<ItemPlan> plans;
    std::vector<cr_status> st;
    std::vector<std::string> errs;
    std::vector<DigitParams> dps;
    std::vector<char> digit_ok;
    std::vector<int> live;  // local indices of the items that reach the device
    bool use_mfma = false, use_bins = false, use_pairs = false;
    int ct = 32, nphase = 0, fallbacks = 0;
    struct Launch {
        int phase, key, tile0, ntiles;
        bool pairs;  // tile pairs (k_reduce_mfma5), else single tiles
    };
    std::vector<Launch> launches;
    std::vector<size_t> comb_first, comb_count;
    size_t h_end = 0, o_items = 0, o_tiles = 0, o_ditems = 0, o_tables = 0, o_cu = 0, o_cg = 0, o_cp = 0, o_vx = 0;
    size_t o_comb = 0, o_msrc = 0, o_malpha = 0, o_err = 0, o_Y = 0, o_hbuf = 0, o_store = 0, o_queue = 0;
    size_t o_psi_dev = 0;
    size_t o_xw = 0;  // streaming kernel: digit planes in global memory
    DevFamily df{};
    hipEvent_t ep = nullptr, epe = nullptr, e0 = nullptr, em = nullptr, e1 = nullptr, edone = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> cev;
    double setup_ms = 0, finish_ms = 0;
    float dev_ms = 0, red_ms = 0, asm_ms = 0, comb_ms = 0, psi_ms = 0;
    void destroy_events() {
        for (hipEvent_t *e : {&ep, &epe, &e0, &em, &e1, &edone})
            if (*e) {
                (void)hipEventDestroy(*e);
                *e = nullptr;
            }
        for (auto &ce : cev) {
            (void)hipEventDestroy(ce.first);
            (void)hipEventDestroy(ce.second);
        }
        cev.clear();
    }
};

// Host setup, plans and the packed device image of one sub-batch (in the
// pinned host half of its arena).
cr_status prepare_sub(BatchCtx &ctx, SubBatch &sb, std::string &msg) {
    auto t0 = std::chrono::steady_clock::now();
    const Family &F = *ctx.F;
    const cr_family *fam = ctx.fam;
    const int count = (int)sb.idx.size(), b = ctx.b, nrt = ctx.nrt, nkb = ctx.nkb, policy = ctx.policy;
    sb.items.assign(count, ItemSetup());
    sb.plans.assign(count, ItemPlan());
    sb.st.assign(count, CR_OK);
    sb.errs.assign(count, std::string());
    sb.dps.assign(count, DigitParams());
    sb.digit_ok.assign(count, 0);
    parallel_for(count, [&](int i) {
        const int g = sb.idx[i];
        sb.st[i] = setup_item(F, ctx.primes[g], ctx.coeffs + (size_t)g * ctx.nco, PrecOpts::from(fam), sb.items[i],
                              sb.errs[i], false, !ctx.device_psi);
        if (sb.st[i] == CR_OK && sb.items[i].b != b) {
            sb.st[i] = CR_ESELFCHECK;
            sb.errs[i] = "basis size differs from the Hodge numbers";
        }
        // depth-first: the device runs Algorithm 3; the chunk count is taken
        // in complete_sub, while the device works
        if (sb.st[i] == CR_OK && policy != CR_POLICY_LEARNED &&
            !plan_item(F, sb.items[i], policy, sb.plans[i], sb.errs[i], policy != CR_POLICY_DEPTH_FIRST))
            sb.st[i] = CR_EINVAL;
        if (sb.st[i] == CR_OK && ctx.want_mfma) {
            ItemSetup &it = sb.items[i];
            int umax = 0;
            for (size_t k = 0; k < it.chain_u.size(); k++) umax = std::max<int>(umax, it.chain_u[k]);
            const u64 wtmax = (u64)umax + (u64)F.g.deg + 1;
            if (ctx.quad || ctx.wide) {
                if (quad_digit_params(it.p, it.M, F.tgt.count, F.nv, wtmax, sb.dps[i]) &&
                    (ctx.quad ? quad_supports_digits(sb.dps[i].D) : wide_supports_digits(sb.dps[i].D))) {
                    it.apack.resize((size_t)nrt * sb.dps[i].D * nkb * 1024);
                    if (!ctx.device_psi)
                        pack_psi_digits(F, it, sb.dps[i], nrt, nkb, it.apack.data(), &ctx.fe->ql);
                    sb.digit_ok[i] = 1;
                }
            } else if (digit_params(it.p, it.M, F.tgt.count, F.nv, wtmax, 10, sb.dps[i]) &&
                       mfma_supports_digits(sb.dps[i].D)) {
                it.apack.resize((size_t)nrt * sb.dps[i].D * nkb * 1024);
                if (!ctx.device_psi)
                    pack_psi_digits(F, it, sb.dps[i], nrt, nkb, it.apack.data(), ctx.use_bins ? &ctx.fe->bl : nullptr);
                sb.digit_ok[i] = 1;
            }
        }
    });
    if (policy == CR_POLICY_LEARNED &&
        !plan_learned(F, sb.items, sb.st, sb.errs, sb.plans, fam->mlp, ctx.stream, sb.fallbacks, msg))
        return CR_EDEVICE;
    sb.live.clear();
    for (int i = 0; i < count; i++)
        if (sb.st[i] == CR_OK) sb.live.push_back(i);
    const int nlive = (int)sb.live.size();
    sb.df = ctx.df;
    DevFamily &df = sb.df;
    sb.use_bins = ctx.use_bins;
    sb.use_mfma = ctx.want_mfma;
    for (int li = 0; li < nlive && sb.use_mfma; li++) sb.use_mfma = sb.digit_ok[sb.live[li]] != 0;
    for (int li = 0; li < nlive && sb.use_mfma && sb.use_bins; li++)
        if (!mfma4_supports(df, sb.dps[sb.live[li]].D)) sb.use_mfma = false;  // packed for the other layout
    if (sb.use_mfma && !sb.use_bins && !ctx.quad && !ctx.wide && policy != CR_POLICY_DEPTH_FIRST) sb.use_mfma = false;
    // tile pairs are chosen per digit count: the items whose digit count the
    // pair kernel takes get their psi digits folded, the others run on single tiles
    sb.use_pairs = sb.use_mfma && sb.use_bins && ctx.pairs && ctx.device_psi;
    auto pairs_for = [&](int D) { return sb.use_pairs && mfma5_supports(df, D); };
    if (sb.use_mfma && !sb.use_bins && !ctx.quad && !ctx.wide && ctx.device_psi)
        sb.use_mfma = false;  // device packing follows the bin layout (or the quad placement)
    if (!sb.use_mfma && ctx.device_psi && ctx.want_mfma) {
        // an item the MFMA kernel cannot take: the VALU kernel reads psi from k_psi directly
    }
    sb.ct = 32;
    if (!sb.use_mfma) {
        while (sb.ct > 1 && reduce_lds_bytes(df, sb.ct) > 64 * 1024) sb.ct /= 2;
        if (reduce_lds_bytes(df, sb.ct) > 64 * 1024) {
            msg = "family too large for the LDS tile";
            return CR_EINVAL;
        }
    }
    sb.launches.clear();
    sb.nphase = 0;
    if (nlive == 0) {
        sb.setup_ms = ms_since(t0);
        return CR_OK;
    }
    const int ct = sb.ct;

    // ---- vectors of every phase in launch order (phase, digit group, item), tiles of ct vectors of one item
    std::vector<int> gkey(nlive, 0), dvals;
    for (int li = 0; li < nlive; li++)
        if (sb.use_mfma && !ctx.quad)  // the quad kernel takes every digit count in one launch
            gkey[li] = sb.dps[sb.live[li]].D + (ctx.wide ? 0 : 100 * sb.dps[sb.live[li]].z32);
    dvals = gkey;
    std::sort(dvals.begin(), dvals.end());
    dvals.erase(std::unique(dvals.begin(), dvals.end()), dvals.end());
    for (int li = 0; li < nlive; li++) sb.nphase = std::max(sb.nphase, (int)sb.plans[sb.live[li]].phase.size());
    const int nphase = sb.nphase;
    std::vector<DevTile> tiles;
    std::vector<std::vector<size_t>> vec0(nlive, std::vector<size_t>(nphase, 0));
    size_t nvec = 0;
    for (int t = 0; t < nphase; t++)
        for (int key : dvals) {
            const int first = (int)tiles.size();
            for (int li = 0; li < nlive; li++) {
                const ItemPlan &pl = sb.plans[sb.live[li]];
                if (gkey[li] != key || t >= (int)pl.phase.size()) continue;
                const auto &ph = pl.phase[t];
                vec0[li][t] = nvec;
                for (int c0 = 0; c0 < (int)ph.size(); c0 += ct) {
                    DevTile tl{};
                    tl.item = li;
                    tl.count = std::min(ct, (int)ph.size() - c0);
                    tl.chain0 = (int32_t)(nvec + c0);
                    tl.steps = ph[c0].pole - ph[c0].pend;
                    tiles.push_back(tl);
                }
                nvec += ph.size();
            }
            if (pairs_for(key % 100) && (int)tiles.size() > first) {
                // pairs of tiles of one item (an odd one out gets an empty partner),
                // longest pairs first
                std::vector<std::pair<DevTile, DevTile>> pr;
                for (size_t k = first; k < tiles.size();) {
                    DevTile a = tiles[k], b = a;
                    b.count = 0;
                    b.steps = 0;
                    if (k + 1 < tiles.size() && tiles[k + 1].item == a.item) {
                        b = tiles[k + 1];
                        k += 2;
                    } else {
                        k += 1;
                    }
                    pr.push_back({a, b});
                }
                std::stable_sort(pr.begin(), pr.end(), [](const std::pair<DevTile, DevTile> &x,
                                                          const std::pair<DevTile, DevTile> &y) {
                    return std::max(x.first.steps, x.second.steps) > std::max(y.first.steps, y.second.steps);
                });
                tiles.resize(first);
                for (auto &q : pr) {
                    tiles.push_back(q.first);
                    tiles.push_back(q.second);
                }
                sb.launches.push_back({t, key, first, (int)pr.size(), true});
                continue;
            }
            // longest tiles first, so that the last wave of workgroups is short
            std::stable_sort(tiles.begin() + first, tiles.end(),
                             [](const DevTile &x, const DevTile &y) { return x.steps > y.steps; });
            if ((int)tiles.size() > first) sb.launches.push_back({t, key, first, (int)tiles.size() - first, false});
        }
    std::vector<int32_t> row0(nlive, 0);
    std::vector<size_t> coef0(nlive, 0), fin0(nlive, 0), apack_off(nlive, 0);
    size_t nrows = 0, ncomb = 0, nmem = 0, nfin_all = 0, ncoef = 0;
    for (int li = 0; li < nlive; li++) {
        const ItemPlan &pl = sb.plans[sb.live[li]];
        row0[li] = (int32_t)nrows;
        nrows += pl.nrows;
        for (auto &cb : pl.comb) ncomb += cb.size();
        nmem += pl.msrc.size();
        fin0[li] = nfin_all;
        for (auto &ph : pl.phase)
            for (auto &v : ph) nfin_all += v.out < 0;
        coef0[li] = ncoef;
        ncoef += (size_t)(sb.items[sb.live[li]].nchain() + b) * b;
    }
    if (nvec >= (size_t)INT32_MAX || nrows >= (size_t)INT32_MAX / 2) {
        msg = "batch too large for 32-bit vector indices";
        return CR_ENOMEM;
    }

    // ---- device layout
    const size_t psi_len = (size_t)F.nsrc * F.tgt.count, rho_len = (size_t)b * F.fin.count;
    const int sdim = ctx.sdim;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    FamilyEntry *fe = ctx.fe;
    sb.o_tables = take(fe->tables.size());
    sb.o_items = take(sizeof(DevItem) * nlive);
    sb.o_tiles = take(sizeof(DevTile) * std::max<size_t>(tiles.size(), 1));
    const bool dpsi = ctx.device_psi;
    const size_t o_psi = take(sb.use_mfma || dpsi ? 0 : 8 * psi_len * nlive);
    if (sb.use_mfma) {
        sb.o_ditems = take(sizeof(DevDigitItem) * nlive);
        if (!dpsi)
            for (int li = 0; li < nlive; li++) apack_off[li] = take(sb.items[sb.live[li]].apack.size());
    }
    const size_t o_rho = take(8 * rho_len * nlive);
    const size_t o_coef = take(8 * ncoef);
    sb.o_cu = take(2 * (size_t)F.nv * nvec);
    sb.o_cg = take(4 * nvec);
    sb.o_cp = take(4 * nvec);
    sb.o_vx = take(sizeof(DevVec) * nvec);
    sb.o_comb = take(sizeof(DevComb) * std::max<size_t>(ncomb, 1));
    sb.o_msrc = take(4 * std::max<size_t>(nmem, 1));
    sb.o_malpha = take(8 * std::max<size_t>(nmem, 1));
    const size_t o_fvec = take(4 * std::max<size_t>(nfin_all, 1));
    const size_t o_frow = take(4 * std::max<size_t>(nfin_all, 1));
    sb.o_err = take(4 * (1 + (size_t)nlive));  // error bits, then one k_psi flag per item
    sb.h_end = off;  // everything above is uploaded
    if (sb.use_mfma && dpsi)
        for (int li = 0; li < nlive; li++) apack_off[li] = take(sb.items[sb.live[li]].apack.size());
    sb.o_queue = take(4 * std::max<size_t>(sb.launches.size(), 1));
    if (sb.use_mfma && ctx.wide) {  // digit planes of the streaming kernel, per workgroup of the persistent grid
        int dmax = 1;
        for (int li = 0; li < nlive; li++) dmax = std::max(dmax, sb.dps[sb.live[li]].D);
        sb.o_xw = take(wide_scratch_bytes(dmax, wide_grid(1 << 30, std::max(1, ctx.fam->grid))));
    }
    sb.o_Y = take(8 * (size_t)b * b * nlive);
    const size_t o_H = take(8 * (size_t)F.fin.count * b * nlive);
    sb.o_hbuf = take(8 * (size_t)F.fin.count * nvec);
    sb.o_store = take(8 * (size_t)sdim * std::max<size_t>(nrows, 1));
    const size_t d_end = off;
    Arena &ar = *ctx.arenas[sb.arena];
    if (!ar.ensure(d_end, sb.o_Y + 8 * (size_t)b * b * nlive)) {
        msg = ar.fixed ? "the sub-batch needs " + std::to_string(d_end) + " bytes of device memory; its slice of the "
                         "static workspace holds " + std::to_string(ar.dev_cap)
                       : "device or pinned host allocation failed";
        return CR_ENOMEM;
    }
    unsigned char *hb = static_cast<unsigned char *>(ar.host);
    unsigned char *db = static_cast<unsigned char *>(ar.dev);
    std::memcpy(hb + sb.o_tables, fe->tables.data(), fe->tables.size());
    df.colmap = reinterpret_cast<const int16_t *>(db + sb.o_tables + fe->off_colmap);
    df.gsrc = reinterpret_cast<const int16_t *>(db + sb.o_tables + fe->off_gsrc);
    df.gw = reinterpret_cast<const int16_t *>(db + sb.o_tables + fe->off_gw);
    df.finmap = reinterpret_cast<const int16_t *>(db + sb.o_tables + fe->off_finmap);
    df.dirs = reinterpret_cast<const int8_t *>(db + sb.o_tables + fe->off_dirs);
    df.finU = reinterpret_cast<const int8_t *>(db + sb.o_tables + fe->off_finU);
    DevItem *hitems = reinterpret_cast<DevItem *>(hb + sb.o_items);
    int16_t *hcu = reinterpret_cast<int16_t *>(hb + sb.o_cu);
    int32_t *hcg = reinterpret_cast<int32_t *>(hb + sb.o_cg);
    int32_t *hcp = reinterpret_cast<int32_t *>(hb + sb.o_cp);
    DevVec *hvx = reinterpret_cast<DevVec *>(hb + sb.o_vx);
    DevComb *hcomb = reinterpret_cast<DevComb *>(hb + sb.o_comb);
    int32_t *hmsrc = reinterpret_cast<int32_t *>(hb + sb.o_msrc);
    uint64_t *hmal = reinterpret_cast<uint64_t *>(hb + sb.o_malpha);
    int32_t *hfvec = reinterpret_cast<int32_t *>(hb + o_fvec);
    int32_t *hfrow = reinterpret_cast<int32_t *>(hb + o_frow);
    // combine entries grouped by the phase that reads them
    sb.comb_first.assign(nphase + 1, 0);
    sb.comb_count.assign(nphase + 1, 0);
    {
        size_t at = 0, mat = 0;
        for (int t = 1; t < nphase; t++) {
            sb.comb_first[t] = at;
            for (int li = 0; li < nlive; li++) {
                const ItemPlan &pl = sb.plans[sb.live[li]];
                if (t >= (int)pl.comb.size()) continue;
                for (const PlanComb &pc : pl.comb[t]) {
                    DevComb &dc = hcomb[at++];
                    dc.row = row0[li] + pc.row;
                    dc.item = li;
                    dc.m0 = (int32_t)mat;
                    for (int j = pc.m0; j < pc.m1; j++) {
                        const int32_t src = pl.msrc[j];
                        hmsrc[mat] = src >= 0 ? row0[li] + src : src;
                        hmal[mat] = pl.malpha[j];
                        mat++;
                    }
                    dc.m1 = (int32_t)mat;
                }
            }
            sb.comb_count[t] = at - sb.comb_first[t];
        }
    }
    parallel_for(nlive, [&](int li) {
        const ItemSetup &it = sb.items[sb.live[li]];
        const ItemPlan &pl = sb.plans[sb.live[li]];
        DevItem &di = hitems[li];
        std::memset(&di, 0, sizeof(di));
        di.q = it.mq.q;
        di.mu = it.mq.mu;
        di.sbits = it.mq.sbits;
        di.b = b;
        di.nchain = it.nchain();
        di.p = it.p;
        di.flag = reinterpret_cast<int32_t *>(db + sb.o_err) + 1 + li;
        if (dpsi) {
            di.psi_out = ctx.psi_dev + psi_len * (size_t)sb.idx[sb.live[li]];
            di.psi = di.psi_out;
        } else {
            di.psi = reinterpret_cast<const uint64_t *>(db + o_psi) + psi_len * li;
        }
        di.rho = reinterpret_cast<const uint64_t *>(db + o_rho) + rho_len * li;
        di.coef = reinterpret_cast<const uint64_t *>(db + o_coef) + coef0[li];
        di.Y = reinterpret_cast<uint64_t *>(db + sb.o_Y) + (size_t)b * b * li;
        di.H = reinterpret_cast<uint64_t *>(db + o_H) + (size_t)F.fin.count * b * li;
        uint64_t *hc = reinterpret_cast<uint64_t *>(hb + o_coef) + coef0[li];
        std::memcpy(hc, it.coef.data(), 8 * it.coef.size());
        std::memset(hc + it.coef.size(), 0, 8 * (size_t)b * b);
        for (int c = 0; c < b; c++) hc[it.coef.size() + (size_t)c * b + c] = 1;
        di.fvec = reinterpret_cast<const int32_t *>(db + o_fvec) + fin0[li];
        di.frow = reinterpret_cast<const int32_t *>(db + o_frow) + fin0[li];
        int nfin = 0;
        for (int t = 0; t < (int)pl.phase.size(); t++) {
            const auto &ph = pl.phase[t];
            for (size_t k = 0; k < ph.size(); k++) {
                const PlanVec &pv = ph[k];
                const size_t g = vec0[li][t] + k;
                for (int i = 0; i < F.nv; i++) hcu[g * F.nv + i] = pv.u[i];
                hcg[g] = pv.gamma;
                hcp[g] = pv.pole;
                hvx[g].pend = pv.pend;
                hvx[g].in = pv.in >= 0 ? row0[li] + pv.in : -1;
                hvx[g].out = pv.out >= 0 ? row0[li] + pv.out : -1;
                hvx[g].dir = pv.dir;
                if (pv.out < 0) {
                    hfvec[fin0[li] + nfin] = (int32_t)g;
                    hfrow[fin0[li] + nfin] = pv.crow;
                    nfin++;
                }
            }
        }
        di.nfin = nfin;
        if (sb.use_mfma) {
            const DigitParams &dp = sb.dps[sb.live[li]];
            DevDigitItem &dd = reinterpret_cast<DevDigitItem *>(hb + sb.o_ditems)[li];
            dd.Bd = dp.Bd;
            dd.Qd = dp.Qd;
            dd.invQ = dp.invQ;
            dd.BHd = dp.BHd;
            dd.invBH = dp.invBH;
            dd.Bh = dp.Bh;
            dd.Bsplit = dp.Bsplit;
            dd.invBsplit = dp.invBsplit;
            dd.bias = dp.bias;
            dd.Qp = dp.Qp;
            dd.q = it.mq.q;
            dd.magic = dp.magic;
            dd.shift = dp.shift;
            dd.B = dp.B;
            dd.halfB = dp.halfB;
            dd.D = dp.D;
            dd.h = dp.h;
            dd.ds = dp.ds;
            dd.z32 = dp.z32;
            dd.fold = sb.use_pairs && mfma5_supports(df, dp.D) ? 1 : 0;
            dd.chain0 = 0;
            dd.nchain = it.nchain();
            dd.apack = reinterpret_cast<const int8_t *>(db + apack_off[li]);
            dd.apack_out = reinterpret_cast<int8_t *>(db + apack_off[li]);
            if (!dpsi) std::memcpy(hb + apack_off[li], it.apack.data(), it.apack.size());
        } else if (!dpsi) {
            std::memcpy(hb + o_psi + 8 * psi_len * li, it.psi.data(), 8 * psi_len);
        }
        std::memcpy(hb + o_rho + 8 * rho_len * li, it.rho.data(), 8 * rho_len);
    });
    std::memcpy(hb + sb.o_tiles, tiles.data(), sizeof(DevTile) * tiles.size());
    std::memset(hb + sb.o_err, 0, 4 * (1 + (size_t)nlive));
    sb.setup_ms = ms_since(t0);
    return CR_OK;
}

// Upload, per phase the combines it reads and its reductions, the assembly,
// and the download of Y and the error flags -- all asynchronous on the stream.
cr_status launch_sub(BatchCtx &ctx, SubBatch &sb, std::string &msg) {
    if (sb.live.empty()) return CR_OK;
    hipStream_t stream = ctx.stream;
    Arena &ar = *ctx.arenas[sb.arena];
    unsigned char *hb = static_cast<unsigned char *>(ar.host);
    unsigned char *db = static_cast<unsigned char *>(ar.dev);
    const DevFamily &df = sb.df;
    const int nlive = (int)sb.live.size(), b = ctx.b;
    (void)hipEventCreate(&sb.e0);
    (void)hipEventCreate(&sb.e1);
    (void)hipEventCreate(&sb.em);
    (void)hipEventCreateWithFlags(&sb.edone, hipEventDisableTiming);
    hipError_t he = hipSuccess;
    if (ctx.device_psi) {
        // upload and (MFMA path) the digits of psi in the kernel's fragment
        // order on the auxiliary stream, behind the call's k_psi launch; this
        // overlaps the reduction of the previous sub-batch (whose arena is the
        // other one); the main stream waits for it before the reductions
        hipStream_t aux = nullptr;
        he = ctx.aux(aux);
        (void)hipEventCreate(&sb.epe);
        if (he == hipSuccess) he = hipMemcpyAsync(db, hb, sb.h_end, hipMemcpyHostToDevice, aux);
        const DevItem *dv = reinterpret_cast<const DevItem *>(db + sb.o_items);
        if (he == hipSuccess && sb.use_mfma)
            he = launch_pack_psi(dv, reinterpret_cast<const DevDigitItem *>(db + sb.o_ditems), nlive,
                                 reinterpret_cast<const int16_t *>(
                                     db + sb.o_tables + (ctx.quad || ctx.wide ? ctx.fe->off_qslot_src : ctx.fe->off_slot_src)),
                                 ctx.nrt,
                                 ctx.nkb, ctx.F->tgt.count, ctx.F->nsrc, sb.use_pairs ? 1 : 0, aux);
        (void)hipEventRecord(sb.epe, aux);
        if (he == hipSuccess) he = hipStreamWaitEvent(stream, sb.epe, 0);
    } else {
        he = hipMemcpyAsync(db, hb, sb.h_end, hipMemcpyHostToDevice, stream);
    }
    (void)hipEventRecord(sb.e0, stream);
    const DevItem *ditems_v = reinterpret_cast<const DevItem *>(db + sb.o_items);
    const int16_t *cu = reinterpret_cast<const int16_t *>(db + sb.o_cu);
    const int32_t *cgp = reinterpret_cast<const int32_t *>(db + sb.o_cg);
    const int32_t *cp = reinterpret_cast<const int32_t *>(db + sb.o_cp);
    const DevVec *vxp = reinterpret_cast<const DevVec *>(db + sb.o_vx);
    uint64_t *storep = reinterpret_cast<uint64_t *>(db + sb.o_store);
    uint64_t *hb64 = reinterpret_cast<uint64_t *>(db + sb.o_hbuf);
    int *errp = reinterpret_cast<int *>(db + sb.o_err);
    // the streaming kernel always runs its persistent form (its digit planes are per workgroup)
    const int mode = sb.use_mfma && ctx.wide ? std::max(1, ctx.fam->launch)
                                             : (sb.use_mfma && (sb.use_bins || ctx.quad) ? ctx.fam->launch : 0);
    const int pgrid = mode > 0 ? std::max(1, ctx.fam->grid) : 0;  // persistent: workgroups per CU
    int *queue = reinterpret_cast<int *>(db + sb.o_queue);
    // the reduction phases (and the combines between them) on stream `rs`
    auto reductions = [&](hipStream_t rs, bool timed) -> hipError_t {
        hipError_t e = hipSuccess;
        if (mode > 0) e = launch_zero_ints(queue, (int)sb.launches.size(), rs);
        for (int t = 0; t < sb.nphase && e == hipSuccess; t++) {
            if (t > 0 && sb.comb_count[t] > 0) {
                hipEvent_t a = nullptr, z = nullptr;
                if (timed) {
                    (void)hipEventCreate(&a);
                    (void)hipEventCreate(&z);
                    (void)hipEventRecord(a, rs);
                }
                e = launch_combine(ditems_v, reinterpret_cast<const DevComb *>(db + sb.o_comb) + sb.comb_first[t],
                                   (int)sb.comb_count[t], reinterpret_cast<const int32_t *>(db + sb.o_msrc),
                                   reinterpret_cast<const uint64_t *>(db + sb.o_malpha), storep, ctx.sdim, rs);
                if (timed) {
                    (void)hipEventRecord(z, rs);
                    sb.cev.push_back({a, z});
                }
            }
            for (size_t li = 0; li < sb.launches.size(); li++) {
                const SubBatch::Launch &L = sb.launches[li];
                if (L.phase != t || e != hipSuccess) continue;
                const DevTile *gt = reinterpret_cast<const DevTile *>(db + sb.o_tiles) + L.tile0;
                if (sb.use_mfma) {
                    const DevDigitItem *ditems = reinterpret_cast<const DevDigitItem *>(db + sb.o_ditems);
                    const int Dg = L.key % 100;
                    const bool z32g = L.key >= 100;
                    if (ctx.quad)
                        e = launch_reduce_quad(df, ditems, gt, L.ntiles, cu, cgp, cp, vxp, storep, hb64,
                                               reinterpret_cast<const uint32_t *>(db + sb.o_tables + ctx.fe->off_qslots),
                                               errp, pgrid, queue + li, rs);
                    else if (ctx.wide)
                        e = launch_reduce_wide(df, ditems, gt, L.ntiles, cu, cgp, cp, vxp, storep, hb64,
                                               reinterpret_cast<const uint32_t *>(db + sb.o_tables + ctx.fe->off_qslots),
                                               errp, Dg, wide_grid(L.ntiles, pgrid),
                                               reinterpret_cast<int8_t *>(db + sb.o_xw), queue + li, rs);
                    else if (L.pairs)
                        e = launch_reduce_mfma5(df, ditems, gt, L.ntiles, cu, cgp, cp, vxp, storep, hb64,
                                                reinterpret_cast<const uint32_t *>(db + sb.o_tables + ctx.fe->off_slots),
                                                errp, Dg, z32g, pgrid, queue + li, rs);
                    else if (sb.use_bins)
                        e = launch_reduce_mfma4(df, ditems, gt, L.ntiles, cu, cgp, cp, vxp, storep, hb64,
                                                reinterpret_cast<const uint32_t *>(db + sb.o_tables + ctx.fe->off_slots),
                                                errp, Dg, z32g, pgrid, queue + li, rs);
                    else
                        e = launch_reduce_mfma(df, ditems, gt, L.ntiles, cu, cgp, cp, hb64, errp, Dg, rs);
                } else {
                    e = launch_reduce(df, ditems_v, gt, L.ntiles, cu, cgp, cp, vxp, storep, hb64, sb.ct, errp, rs);
                }
            }
        }
        return e;
    };
    if (he == hipSuccess && mode == 2) {
        // signature of every launch parameter: an identical one replays the cached graph
        std::string sig = std::to_string((uintptr_t)db) + ":" + std::to_string(sb.nphase) + ":" + std::to_string(pgrid);
        for (auto &L : sb.launches)
            sig += "|" + std::to_string(L.phase) + "," + std::to_string(L.key) + "," + std::to_string(L.tile0) + "," +
                   std::to_string(L.ntiles) + (L.pairs ? "p" : "s");
        for (int t = 0; t < sb.nphase; t++) sig += "/" + std::to_string(sb.comb_first[t]) + "," + std::to_string(sb.comb_count[t]);
        for (size_t o : {sb.o_items, sb.o_tiles, sb.o_ditems, sb.o_tables, sb.o_cu, sb.o_cg, sb.o_cp, sb.o_vx,
                         sb.o_comb, sb.o_msrc, sb.o_malpha, sb.o_err, sb.o_hbuf, sb.o_store, sb.o_queue, sb.o_xw})
            sig += ";" + std::to_string(o);
        hipGraphExec_t exec = nullptr;
        auto f = g_graphs.find(sig);
        if (f != g_graphs.end()) {
            exec = f->second;
        } else {
            if (!g_capture) he = hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking);
            hipGraph_t graph = nullptr;
            if (he == hipSuccess) he = hipStreamBeginCapture(g_capture, hipStreamCaptureModeRelaxed);
            if (he == hipSuccess) {
                hipError_t ec = reductions(g_capture, false);
                he = hipStreamEndCapture(g_capture, &graph);
                if (he == hipSuccess) he = ec;
            }
            if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (he == hipSuccess) {
                if (g_graphs.size() >= 16) clear_graphs();
                g_graphs.emplace(sig, exec);
            }
        }
        if (he == hipSuccess) he = hipGraphLaunch(exec, stream);
    } else if (he == hipSuccess) {
        he = reductions(stream, true);
    }
    (void)hipEventRecord(sb.em, stream);
    if (he == hipSuccess) he = launch_assemble(df, ditems_v, nlive, hb64, stream);
    (void)hipEventRecord(sb.e1, stream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(hb + sb.o_Y, db + sb.o_Y, 8 * (size_t)b * b * nlive, hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(hb + sb.o_err, db + sb.o_err, 4 * (1 + (size_t)nlive), hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess) he = hipEventRecord(sb.edone, stream);
    if (he != hipSuccess) {
        msg = std::string("HIP error: ") + hipGetErrorString(he);
        return CR_EDEVICE;
    }
    return CR_OK;
}

// Waits for the sub-batch, then unscales and recovers Q(T) of its items.
cr_status complete_sub(BatchCtx &ctx, SubBatch &sb, std::vector<cr_status> &st, std::vector<std::string> &errs,
                       std::string &msg) {
    const int count = (int)sb.idx.size(), b = ctx.b;
    for (int i = 0; i < count; i++) {
        st[sb.idx[i]] = sb.st[i];
        errs[sb.idx[i]] = sb.errs[i];
    }
    if (sb.live.empty()) return CR_OK;
    if (ctx.policy == CR_POLICY_DEPTH_FIRST)
        parallel_for((int)sb.live.size(), [&](int li) {
            const int i = sb.live[li];
            sb.plans[i].chunks = std::max<int64_t>(0, depth_first_chunks(*ctx.F, sb.items[i]));
        });
    // edone follows the downloads of this sub-batch only (later sub-batches may still run)
    hipError_t he = hipEventSynchronize(sb.edone);
    if (he == hipSuccess) {
        (void)hipEventElapsedTime(&sb.dev_ms, sb.e0, sb.e1);
        (void)hipEventElapsedTime(&sb.red_ms, sb.e0, sb.em);
        (void)hipEventElapsedTime(&sb.asm_ms, sb.em, sb.e1);
        if (sb.ep) (void)hipEventElapsedTime(&sb.psi_ms, sb.ep, sb.epe);
        for (auto &ce : sb.cev) {
            float x = 0;
            (void)hipEventElapsedTime(&x, ce.first, ce.second);
            sb.comb_ms += x;
        }
    }
    sb.destroy_events();
    if (he != hipSuccess) {
        msg = std::string("HIP error: ") + hipGetErrorString(he);
        return CR_EDEVICE;
    }
    unsigned char *hb = static_cast<unsigned char *>(ctx.arenas[sb.arena]->host);
    int derr;
    std::memcpy(&derr, hb + sb.o_err, 4);
    if (derr) {
        msg = "device reduction invariant violated (code " + std::to_string(derr) + ")";
        return CR_ESELFCHECK;
    }
    const int32_t *flags = reinterpret_cast<const int32_t *>(hb + sb.o_err) + 1;
    auto t2 = std::chrono::steady_clock::now();
    const uint64_t *Yh = reinterpret_cast<const uint64_t *>(hb + sb.o_Y);
    const Outputs &o = ctx.out;
    parallel_for((int)sb.live.size(), [&](int li) {
        const int i = sb.live[li], g = sb.idx[i];
        const size_t bb = (size_t)b * b;
        if (flags[li] || (ctx.psi_flags && ctx.psi_flags[g])) {
            // J_S not surjective mod p: f is singular (S = all) or not S-smooth (Definition 3.1)
            const bool all = ctx.F->nS == ctx.F->nv;
            st[g] = all ? CR_ESINGULAR : CR_ENOT_S_SMOOTH;
            errs[g] = all ? "J_S is not surjective mod p (no unit pivot): f is singular mod p"
                          : "J_S is not surjective mod p (no unit pivot): f is not S-smooth";
            return;
        }
        st[g] = finish_item(*ctx.F, sb.items[i], Yh + bb * li, o.frob + bb * g, o.col_pole + (size_t)b * g,
                            o.col_prec + (size_t)b * g, o.lpoly + (size_t)4 * (b + 1) * g, errs[g]);
        if (o.frob_scaled) std::memcpy(o.frob_scaled + bb * g, Yh + bb * li, 8 * bb);
    });
    sb.finish_ms = ms_since(t2);
    return CR_OK;
}

}  // namespace

namespace crf {
bool trace_item(const cr_family *fam, int p, const uint32_t *coeffs, std::vector<CandRow> &rows, std::string &err,
                cr_status &st) {
    if (!check_family(fam, err)) {
        st = CR_EINVAL;
        return false;
    }
    FamilyEntry *fe;
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        fe = get_family(fam, err);
    }
    if (!fe) {
        st = CR_EINVAL;
        return false;
    }
    ItemSetup it;
    st = setup_item(fe->fam, p, coeffs, PrecOpts::from(fam), it, err);
    if (st != CR_OK) return false;
    PChunkPlanner pc;
    if (!pc.init(fe->fam, it, CR_POLICY_P_CHUNK, err)) {
        st = CR_EINVAL;
        return false;
    }
    while (pc.begin_phase()) {
        pc.candidates(rows);
        std::vector<int32_t> none(pc.act.size(), -1);
        if (!pc.end_phase(none, err)) {
            st = CR_ESELFCHECK;
            return false;
        }
    }
    return true;
}
}  // namespace crf

extern "C" {

const char *cr_last_error(void) { return g_err.c_str(); }

cr_status cr_query_dims(int32_t nvars, int32_t degree, int32_t *ncoeff, int32_t *s, int32_t *b) {
    if (nvars < 3 || nvars > kMaxVars || degree < 2) return fail(CR_EINVAL, "unsupported nvars/degree");
    const int n = nvars - 1;
    if (ncoeff) *ncoeff = (int32_t)count_monomials(nvars, degree);
    if (s) *s = (int32_t)count_monomials(nvars, degree * n - n);
    if (b) {
        long long t = 0;
        for (int m = 1; m <= n; m++) t += hodge_size(nvars, degree, m);
        *b = (int32_t)t;
    }
    return CR_OK;
}

cr_status cr_monomials(int32_t nvars, int32_t degree, int32_t *exps) {
    if (nvars < 3 || nvars > kMaxVars || degree < 2 || !exps) return fail(CR_EINVAL, "bad arguments");
    MonoSpace sp;
    sp.init(nvars, degree);
    for (size_t k = 0; k < sp.exps.size(); k++) exps[k] = sp.exps[k];
    return CR_OK;
}

cr_status cr_precision(const cr_family *fam, int32_t p, int32_t *r, int32_t *n_series, int32_t *M) {
    std::string err;
    if (!check_family(fam, err)) return fail(CR_EINVAL, err);
    const int n = fam->nvars - 1;
    std::vector<int> hodge(n);
    for (int m = 1; m <= n; m++) hodge[m - 1] = (int)hodge_size(fam->nvars, fam->degree, m);
    int rr, MM;
    std::vector<int> Nm;
    if (!choose_precision(p, n, hodge, PrecOpts::from(fam), rr, Nm, MM, err)) return fail(CR_EINVAL, err);
    if (r) *r = rr;
    if (n_series) *n_series = *std::max_element(Nm.begin(), Nm.end());
    if (M) *M = MM;
    return CR_OK;
}

cr_status cr_residue_words(const cr_family *fam, int32_t p, int32_t *words) {
    if (!words) return fail(CR_EINVAL, "null pointer");
    int32_t r, N, M;
    cr_status st = cr_precision(fam, p, &r, &N, &M);
    if (st != CR_OK) return st;
    if (p < 2) return fail(CR_ENOTPRIME, "p is not prime");
    long double q = 1;
    for (int k = 0; k < M; k++) q *= p;
    if (q >= std::ldexp(1.0L, 55)) return fail(CR_EPRECISION, "p^M exceeds the 55-bit residues of this build");
    *words = 1;
    return CR_OK;
}

cr_status cr_check_smooth(const cr_family *fam, int32_t p, const uint32_t *coeffs, int32_t *smooth) {
    std::string err;
    if (!check_family(fam, err) || !coeffs || !smooth) return fail(CR_EINVAL, err.empty() ? "null pointer" : err);
    FamilyEntry *fe;
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        fe = get_family(fam, err);
    }
    if (!fe) return fail(CR_EINVAL, err);
    ItemSetup it;
    cr_status st = setup_item(fe->fam, p, coeffs, PrecOpts::from(fam), it, err, true);
    if (st == CR_ESINGULAR || st == CR_ENOT_S_SMOOTH) {
        *smooth = 0;
        return CR_OK;
    }
    if (st != CR_OK) return fail(st, err);
    *smooth = 1;
    return CR_OK;
}

cr_status cr_policy_cost(const cr_family *fam, int32_t p, const uint32_t *coeffs, cr_stats *stats) {
    std::string err;
    if (!check_family(fam, err) || !coeffs || !stats) return fail(CR_EINVAL, err.empty() ? "null pointer" : err);
    FamilyEntry *fe;
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        fe = get_family(fam, err);
    }
    if (!fe) return fail(CR_EINVAL, err);
    auto t0 = std::chrono::steady_clock::now();
    ItemSetup it;
    cr_status st = setup_item(fe->fam, p, coeffs, PrecOpts::from(fam), it, err);
    if (st != CR_OK) return fail(st, err);
    ItemPlan plan;
    if (!plan_item(fe->fam, it, fam->policy, plan, err)) return fail(CR_EINVAL, err);
    std::memset(stats, 0, sizeof(*stats));
    stats->start_blocks = it.nchain();
    stats->column_steps = plan.column_steps;
    stats->chunks = plan.chunks;
    stats->vectors = plan.vectors;
    stats->merged_terms = plan.merged_terms;
    stats->combined_groups = plan.combined_groups;
    stats->phases = (int32_t)plan.phase.size();
    stats->policy = fam->policy;
    stats->engine = -1;
    stats->setup_ms = ms_since(t0);
    return CR_OK;
}

cr_status cr_release(void) {
    std::lock_guard<std::mutex> lk(g_mutex);
    clear_graphs();
    for (Arena &a : g_arenas) a.release();
    g_psi_arena.release();
    return CR_OK;
}

cr_status cr_set_allocator(cr_alloc_fn alloc, cr_free_fn free_, void *ctx) {
    if ((alloc == nullptr) != (free_ == nullptr)) return fail(CR_EINVAL, "cr_set_allocator needs both hooks or neither");
    std::lock_guard<std::mutex> lk(g_mutex);
    // cached graphs hold the old workspaces' addresses
    clear_graphs();
    for (Arena &a : g_arenas) a.release();
    g_psi_arena.release();
    return set_allocator(alloc, free_, ctx);
}

// psi of every item of a call in one k_psi launch on the auxiliary stream
// (J_S is built on the device from the coefficients), started before the
// first sub-batch's host setup.  Items whose prime the setup will reject get
// q = 0 and are skipped by the kernel.
cr_status start_psi_all(BatchCtx &ctx, int count, std::string &msg) {
    const Family &F = *ctx.F;
    const size_t psi_len = (size_t)F.nsrc * F.tgt.count;
    const int nco = ctx.nco, n = F.n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const size_t o_jtab = take(4 * F.jtab.size());
    const size_t o_coef = take(4 * (size_t)count * nco);
    const size_t o_items = take(sizeof(DevItem) * count);
    const size_t o_flags = take(4 * (size_t)count);
    const size_t h_end = off;
    const size_t o_psi = take(8 * psi_len * count);
    // [J | I] of every item, for the global-memory elimination
    const size_t o_work =
        ctx.psi_global || ctx.psi_multi ? take(8 * (size_t)F.tgt.count * (F.nsrc + F.tgt.count) * count) : 0;
    const size_t o_book = ctx.psi_multi ? take(psi_book_bytes(F.tgt.count, F.nsrc) * count) : 0;
    Arena &ar = *ctx.psi_arena;
    if (!ar.ensure(off, h_end)) {
        msg = ar.fixed ? "the right inverses of J_S need " + std::to_string(off) + " bytes of device memory; the "
                         "static workspace holds " + std::to_string(ar.dev_cap)
                       : "device or pinned host allocation failed";
        return CR_ENOMEM;
    }
    ctx.psi_bytes = off;
    unsigned char *hb = static_cast<unsigned char *>(ar.host);
    unsigned char *db = static_cast<unsigned char *>(ar.dev);
    std::memcpy(hb + o_jtab, F.jtab.data(), 4 * F.jtab.size());
    std::memcpy(hb + o_coef, ctx.coeffs, 4 * (size_t)count * nco);
    std::memset(hb + o_flags, 0, 4 * (size_t)count);
    std::vector<int> hodge(n);
    for (int m = 1; m <= n; m++) hodge[m - 1] = (int)hodge_size(F.nv, F.d, m);
    std::map<int, ModQ> mods;  // prime -> q = p^M (0 when the setup rejects the prime)
    DevItem *hit = reinterpret_cast<DevItem *>(hb + o_items);
    for (int g = 0; g < count; g++) {
        const int p = ctx.primes[g];
        auto m = mods.find(p);
        if (m == mods.end()) {
            ModQ mq;
            bool prime = p >= 2;
            for (int t = 2; t * t <= p && prime; t++) prime = p % t != 0;
            int rr, MM;
            std::vector<int> NN;
            std::string e2;
            if (prime && p >= 7 && p < 50 && p > n && F.d % p != 0 &&
                choose_precision(p, n, hodge, PrecOpts::from(ctx.fam), rr, NN, MM, e2)) {
                u64 q = 1;
                for (int k = 0; k < MM; k++) q *= (u64)p;
                mq.init(q);
            }
            m = mods.emplace(p, mq).first;
        }
        DevItem &di = hit[g];
        std::memset(&di, 0, sizeof(di));
        di.q = m->second.q;
        di.mu = m->second.mu;
        di.sbits = m->second.sbits;
        di.p = p;
        di.fcoef = reinterpret_cast<const uint32_t *>(db + o_coef) + (size_t)g * nco;
        di.psi_out = reinterpret_cast<uint64_t *>(db + o_psi) + psi_len * g;
        di.flag = reinterpret_cast<int32_t *>(db + o_flags) + g;
    }
    hipStream_t aux = nullptr;
    hipError_t he = ctx.aux(aux);
    (void)hipEventCreate(&ctx.psi_t0);
    (void)hipEventCreate(&ctx.psi_done);
    if (he == hipSuccess) he = hipMemcpyAsync(db, hb, h_end, hipMemcpyHostToDevice, aux);
    (void)hipEventRecord(ctx.psi_t0, aux);
    if (he == hipSuccess && ctx.psi_multi)
        he = launch_psi_multi(reinterpret_cast<const DevItem *>(db + o_items), count, F.tgt.count, F.nsrc,
                              reinterpret_cast<const int32_t *>(db + o_jtab), reinterpret_cast<uint64_t *>(db + o_work),
                              db + o_book, aux);
    else if (he == hipSuccess && ctx.psi_global)
        he = launch_psi_global(reinterpret_cast<const DevItem *>(db + o_items), count, F.tgt.count, F.nsrc,
                               reinterpret_cast<const int32_t *>(db + o_jtab),
                               reinterpret_cast<uint64_t *>(db + o_work), aux);
    else if (he == hipSuccess)
        he = launch_psi(reinterpret_cast<const DevItem *>(db + o_items), count, F.tgt.count, F.nsrc,
                        reinterpret_cast<const int32_t *>(db + o_jtab), aux);
    if (he == hipSuccess)
        he = hipMemcpyAsync(hb + o_flags, db + o_flags, 4 * (size_t)count, hipMemcpyDeviceToHost, aux);
    (void)hipEventRecord(ctx.psi_done, aux);
    if (he != hipSuccess) {
        msg = std::string("HIP error: ") + hipGetErrorString(he);
        return CR_EDEVICE;
    }
    ctx.psi_dev = reinterpret_cast<uint64_t *>(db + o_psi);
    ctx.psi_flags = reinterpret_cast<const int32_t *>(hb + o_flags);
    return CR_OK;
}

}  // extern "C"

namespace {

hipError_t static_ws(void **ptr, size_t *bytes);

// cr_frobenius_batch, and with noalloc its allocation-free variant (fixed
// arenas in the static workspace, every stream operation on the caller's
// stream, no graph capture, no model buffers).
cr_status frobenius_batch(const cr_family *fam, int32_t count, const int32_t *primes, const uint32_t *coeffs,
                          uint64_t *frob, uint64_t *frob_scaled, int32_t *col_pole, int32_t *col_prec, int64_t *lpoly,
                          int32_t *item_status, cr_stats *stats, void *hip_stream, bool noalloc) {
    std::string err;
    if (!check_family(fam, err)) return fail(CR_EINVAL, err);
    if (count < 0 || (count > 0 && (!primes || !coeffs || !frob || !col_pole || !col_prec || !lpoly)))
        return fail(CR_EINVAL, "null output or input pointer");
    if (count == 0) return CR_OK;
    if (fam->policy == CR_POLICY_LEARNED && !fam->mlp) return fail(CR_EINVAL, "CR_POLICY_LEARNED needs a model (cr_family.mlp)");
    if (noalloc && fam->policy == CR_POLICY_LEARNED)
        return fail(CR_EINVAL, "the allocation-free entry point does not run CR_POLICY_LEARNED (the network's row "
                               "buffers grow with the batch)");
    if (noalloc && fam->launch == 2)
        return fail(CR_EINVAL, "the allocation-free entry point does not capture graphs (launch mode 2)");
    std::lock_guard<std::mutex> lk(g_mutex);
    BatchCtx ctx;
    if (!ctx.init(fam, primes, coeffs, reinterpret_cast<hipStream_t>(hip_stream), err)) return fail(CR_EINVAL, err);
    ctx.out = {frob, frob_scaled, col_pole, col_prec, lpoly};
    Arena fixed[kArenas], fixed_psi;
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    if (noalloc) {
        void *wp = nullptr;
        const hipError_t he = static_ws(&wp, &ws_bytes);
        if (he != hipSuccess) return fail(CR_EDEVICE, std::string("static workspace: ") + hipGetErrorString(he));
        ws = static_cast<unsigned char *>(wp);
        ctx.noalloc = true;
        fixed_psi.bind(ws, ws_bytes);
        ctx.psi_arena = &fixed_psi;
        for (int k = 0; k < kArenas; k++) ctx.arenas[k] = &fixed[k];
    }
    // Sub-batches: the host prepares sub-batch k + 1 while the device reduces
    // sub-batch k.  Sizes follow the width P of the host pool (each item's
    // setup is one task).  Where an item's host setup is about as long as its
    // share of the device work (quartic K3 surfaces: one pool round of setup,
    // 64 ms, against 82 ms of reduction for P = 16 surfaces), every
    // sub-batch is one round, so that the setup of the next one always hides
    // behind the reduction of the current one (64 K3 surfaces: 401 against
    // 446-458 ms per call with a second sub-batch of two rounds).  For plane
    // curves (setup well under a millisecond per item) the device time lost
    // in launch tails outweighs the wait for a larger first sub-batch: the
    // sub-batches grow by two rounds each, 2P, 4P, 6P, ... (256 plane
    // quintics: 32, 64, 96 and 64 curves, 4 launches instead of 9, 13.7
    // against 14.8 ms; the mixed-prime batch 24.3 against 26.0 ms with 2P
    // then 4P).  The allocation-free entry point keeps one round, then two
    // (its sub-batches share one fixed workspace).
    const int P = Pool::get().width();
    const bool small = ctx.F->g.count <= 64;
    std::vector<int> cut{0};
    if (count <= (noalloc ? 2 * P : (small ? 3 * P : P))) {
        cut.push_back(count);
    } else {
        for (int k = 0; cut.back() < count; k++) {
            const int size = noalloc ? (k == 0 ? P : 2 * P) : (small ? 2 * P * (k + 1) : P);
            cut.push_back(std::min(count, cut.back() + size));
        }
    }
    const int S = (int)cut.size() - 1;
    std::vector<SubBatch> sub(S);
    for (int k = 0; k < S; k++) {
        for (int i = cut[k]; i < cut[k + 1]; i++) sub[k].idx.push_back(i);
        sub[k].arena = noalloc ? 0 : k % kArenas;
    }
    std::vector<cr_status> st(count, CR_OK);
    std::vector<std::string> errs(count);
    cr_status fatal = CR_OK;
    std::string fatal_msg;
    auto drop_psi = [&]() {
        if (ctx.psi_t0) (void)hipEventDestroy(ctx.psi_t0);
        if (ctx.psi_done) (void)hipEventDestroy(ctx.psi_done);
        ctx.psi_t0 = ctx.psi_done = nullptr;
    };
    // the call's psi launch only if some item can pass the setup (a prime in
    // range, coefficients reduced mod p): invalid input is reported as such
    bool any_valid = false;
    for (int g = 0; g < count && !any_valid; g++) {
        const int p = primes[g];
        bool ok = p >= 7 && p < 50;
        for (int t = 2; t * t <= p && ok; t++) ok = p % t != 0;
        for (int k = 0; k < ctx.nco && ok; k++) ok = coeffs[(size_t)g * ctx.nco + k] < (uint32_t)p;
        any_valid = ok;
    }
    if (ctx.device_psi && any_valid) {
        fatal = start_psi_all(ctx, count, fatal_msg);
        if (fatal != CR_OK) {
            if (g_aux) (void)hipStreamSynchronize(g_aux);
            drop_psi();
            return fail(fatal, fatal_msg);
        }
    }
    // Without the workspace every sub-batch has its own arena of two, and
    // complete(k - 1) releases the arena that sub-batch k + 1 reuses; with it,
    // one arena (what the call's psi leaves of the workspace) serves every
    // sub-batch in turn, each completed before the next is prepared.
    const int lag = noalloc ? 0 : kArenas - 1;
    if (noalloc) {
        const size_t used = align256(ctx.psi_bytes);
        fixed[0].bind(ws + used, used < ws_bytes ? ws_bytes - used : 0);
    }
    auto stop_all = [&](int upto) {  // drain the device before reporting a failure
        (void)hipStreamSynchronize(ctx.stream);
        if (g_aux) (void)hipStreamSynchronize(g_aux);
        for (int k = 0; k <= upto && k < S; k++) sub[k].destroy_events();
    };
    for (int k = 0; k < S && fatal == CR_OK; k++) {
        fatal = prepare_sub(ctx, sub[k], fatal_msg);
        if (fatal == CR_OK) fatal = launch_sub(ctx, sub[k], fatal_msg);
        if (fatal == CR_OK && k >= lag) fatal = complete_sub(ctx, sub[k - lag], st, errs, fatal_msg);
        if (fatal != CR_OK) stop_all(k);
    }
    for (int k = std::max(0, S - lag); k < S && fatal == CR_OK; k++)
        fatal = complete_sub(ctx, sub[k], st, errs, fatal_msg);
    if (fatal != CR_OK) {
        stop_all(S - 1);
        drop_psi();
        return fail(fatal, fatal_msg);
    }
    float psi_all_ms = 0;
    if (ctx.psi_t0 && ctx.psi_done) (void)hipEventElapsedTime(&psi_all_ms, ctx.psi_t0, ctx.psi_done);
    drop_psi();
    cr_status first = CR_OK;
    for (int i = 0; i < count; i++) {
        if (item_status) item_status[i] = st[i];
        if (st[i] != CR_OK && first == CR_OK) {
            first = st[i];
            g_err = "item " + std::to_string(i) + ": " + errs[i];
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->engine = -1;
        stats->policy = fam->policy;
        for (auto &sb : sub) {
            for (int li = 0; li < (int)sb.live.size(); li++) {
                const ItemPlan &pl = sb.plans[sb.live[li]];
                stats->start_blocks += sb.items[sb.live[li]].nchain();
                stats->column_steps += pl.column_steps;
                stats->chunks += pl.chunks;
                stats->vectors += pl.vectors;
                stats->merged_terms += pl.merged_terms;
                stats->combined_groups += pl.combined_groups;
            }
            stats->setup_ms += sb.setup_ms;
            stats->device_ms += sb.dev_ms + sb.psi_ms;
            stats->psi_ms += sb.psi_ms;
            stats->reduce_ms += sb.red_ms - sb.comb_ms;
            stats->combine_ms += sb.comb_ms;
            stats->assemble_ms += sb.asm_ms;
            stats->finish_ms += sb.finish_ms;
            stats->phases = std::max(stats->phases, sb.nphase);
            stats->reduce_launches += (int64_t)sb.launches.size();
            stats->fallbacks += sb.fallbacks;
            if (!sb.live.empty()) {
                bool any_pairs = false;
                for (auto &L : sb.launches) any_pairs = any_pairs || L.pairs;
                const int e = sb.use_mfma ? (ctx.quad ? 4 : ctx.wide ? 5 : (any_pairs ? 0 : (sb.use_bins ? 3 : 2))) : 1;
                // a sub-batch that fell back to the VALU kernel makes the call report it
                if (stats->engine < 0 || e == 1) stats->engine = e;
            }
        }
        if (stats->engine < 0) stats->engine = 0;
        stats->psi_ms += psi_all_ms;
        stats->device_ms += psi_all_ms;
    }
    auto spent = std::make_shared<std::vector<SubBatch>>(std::move(sub));
    Reaper::get().post([spent]() mutable { spent.reset(); });
    return first;
}

}  // namespace

namespace crf {
hipError_t static_workspace(void **ptr, size_t *bytes);
}

namespace {
hipError_t static_ws(void **ptr, size_t *bytes) { return crf::static_workspace(ptr, bytes); }
}  // namespace

extern "C" {

cr_status cr_frobenius_batch(const cr_family *fam, int32_t count, const int32_t *primes, const uint32_t *coeffs,
                             uint64_t *frob, uint64_t *frob_scaled, int32_t *col_pole, int32_t *col_prec,
                             int64_t *lpoly, int32_t *item_status, cr_stats *stats, void *hip_stream) {
    return frobenius_batch(fam, count, primes, coeffs, frob, frob_scaled, col_pole, col_prec, lpoly, item_status,
                           stats, hip_stream, false);
}

cr_status cr_frobenius_batch_noalloc(const cr_family *fam, int32_t count, const int32_t *primes,
                                     const uint32_t *coeffs, uint64_t *frob, uint64_t *frob_scaled, int32_t *col_pole,
                                     int32_t *col_prec, int64_t *lpoly, int32_t *item_status, cr_stats *stats,
                                     void *hip_stream) {
    return frobenius_batch(fam, count, primes, coeffs, frob, frob_scaled, col_pole, col_prec, lpoly, item_status,
                           stats, hip_stream, true);
}

cr_status cr_frobenius(const cr_family *fam, int32_t p, const uint32_t *coeffs, uint64_t *frob, uint64_t *frob_scaled,
                       int32_t *col_pole, int32_t *col_prec, int64_t *lpoly, cr_stats *stats, void *hip_stream) {
    int32_t st_item = CR_OK;
    const int32_t primes[1] = {p};
    cr_status st = cr_frobenius_batch(fam, 1, primes, coeffs, frob, frob_scaled, col_pole, col_prec, lpoly, &st_item,
                                      stats, hip_stream);
    return st != CR_OK ? st : (cr_status)st_item;
}

}  // extern "C"

namespace {

std::string g_tune_cache;  // file of persisted autotuner results ("" = none)

// Key of a tuned batch: family, count, the multiset of primes, device.
std::string tune_key(const cr_family *fam, int32_t count, const int32_t *primes) {
    std::map<int, int> hist;
    for (int i = 0; i < count; i++) hist[primes[i]]++;
    std::string k = std::to_string(fam->nvars) + "," + std::to_string(fam->degree) + "," + std::to_string(fam->s_mask) +
                    "," + std::to_string(fam->r) + "," + std::to_string(fam->n_series) + "," + std::to_string(fam->M) +
                    ",n=" + std::to_string(count) + ",p=";
    for (auto &h : hist) k += std::to_string(h.first) + "x" + std::to_string(h.second) + ".";
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        k += std::string(",") + prop.gcnArchName + "/" + std::to_string(prop.multiProcessorCount);
    for (char &ch : k)
        if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
    return k;
}

bool tune_lookup(const std::string &key, cr_tuning *out) {
    if (g_tune_cache.empty()) return false;
    FILE *f = std::fopen(g_tune_cache.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[768];
        int pol, lm, eng, grid;
        double ms;
        if (std::sscanf(line, "%767s %d %d %d %d %lf", k, &pol, &lm, &eng, &grid, &ms) == 6 && key == k) {
            out->best_policy = pol;  // the last entry for a key wins
            out->best_launch = lm;
            out->best_engine = eng;
            out->best_grid = grid;
            out->best_ms = ms;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const std::string &key, const cr_tuning *t) {
    if (g_tune_cache.empty()) return;
    FILE *f = std::fopen(g_tune_cache.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %.4f\n", key.c_str(), t->best_policy, t->best_launch, t->best_engine, t->best_grid,
                 t->best_ms);
    std::fclose(f);
}

}  // namespace

extern "C" {

cr_status cr_autotune_cache(const char *path) {
    std::lock_guard<std::mutex> lk(g_mutex);
    g_tune_cache = path ? path : "";
    return CR_OK;
}

cr_status cr_autotune(const cr_family *fam, int32_t count, const int32_t *primes, const uint32_t *coeffs,
                      int32_t trials, cr_tuning *out, void *hip_stream) {
    std::string err;
    if (!check_family(fam, err) || !out || count <= 0 || trials < 1 || !primes || !coeffs)
        return fail(CR_EINVAL, err.empty() ? "bad arguments" : err);
    int32_t nco, s_dim, b;
    cr_query_dims(fam->nvars, fam->degree, &nco, &s_dim, &b);
    std::vector<uint64_t> frob((size_t)count * b * b);
    std::vector<int32_t> pole((size_t)count * b), prec((size_t)count * b), ist(count);
    std::vector<int64_t> lp((size_t)count * (b + 1) * 4);
    std::memset(out, 0, sizeof(*out));
    for (double &x : out->ms) x = -1;
    for (double &x : out->shape_ms) x = -1;
    out->best_ms = -1;
    std::string key;
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        key = tune_key(fam, count, primes);
        if (tune_lookup(key, out)) {
            out->from_cache = 1;
            return CR_OK;
        }
    }
    // mean wall time of `trials` calls after one warm-up call; -1 if a call
    // fails, or (for an explicit engine) ran another kernel than the one asked
    // for.  Items whose Q(T) is out of reach of an overridden precision
    // (CR_EPRECISION after the reduction ran) do not make the call a failure.
    auto time_cfg = [&](const cr_family &f) -> double {
        double tot = 0;
        for (int r = 0; r <= trials; r++) {
            cr_stats st{};
            auto t0 = std::chrono::steady_clock::now();
            cr_status cs = cr_frobenius_batch(&f, count, primes, coeffs, frob.data(), nullptr, pole.data(),
                                              prec.data(), lp.data(), ist.data(), &st, hip_stream);
            bool ran = cs == CR_OK;
            if (!ran && cs == CR_EPRECISION && st.column_steps > 0) {
                ran = true;
                for (int i = 0; i < count; i++) ran = ran && (ist[i] == CR_OK || ist[i] == CR_EPRECISION);
            }
            if (!ran || (f.engine != 0 && st.engine != f.engine)) return -1;
            if (r > 0) tot += ms_since(t0);
        }
        return tot / trials;
    };
    std::vector<int> pols = {CR_POLICY_DEPTH_FIRST, CR_POLICY_P_CHUNK, CR_POLICY_VAR_BY_VAR};
    if (fam->mlp) pols.push_back(CR_POLICY_LEARNED);
    for (int pol : pols)
        for (int lm = 0; lm < 3; lm++) {
            cr_family f = *fam;
            f.policy = pol;
            f.launch = lm;
            if (!check_family(&f, err)) continue;
            const double ms = time_cfg(f);
            if (ms < 0) continue;
            out->ms[pol * 3 + lm] = ms;
            if (out->best_ms < 0 || ms < out->best_ms) {
                out->best_ms = ms;
                out->best_policy = pol;
                out->best_launch = lm;
                out->best_engine = fam->engine;
                out->best_grid = std::max(1, fam->grid);
            }
        }
    if (out->best_ms < 0) return fail(CR_EINVAL, "no configuration ran: " + g_err);
    // kernel shapes for the best (policy, launch)
    static const int shapes[8][2] = {{0, 1}, {0, 2}, {3, 1}, {3, 2}, {2, 1}, {4, 1}, {4, 2}, {1, 1}};
    for (int k = 0; k < 8; k++) {
        cr_family f = *fam;
        f.policy = out->best_policy;
        f.launch = out->best_launch;
        f.engine = shapes[k][0];
        f.grid = shapes[k][1];
        if (f.launch == 0 && f.grid > 1) continue;  // the grid only shapes persistent launches
        if (!check_family(&f, err)) continue;
        const double ms = time_cfg(f);
        out->shape_ms[k] = ms;
        if (ms >= 0 && ms < out->best_ms) {
            out->best_ms = ms;
            out->best_engine = f.engine;
            out->best_grid = f.grid;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        tune_store(key, out);
    }
    return CR_OK;
}

}  // extern "C"
