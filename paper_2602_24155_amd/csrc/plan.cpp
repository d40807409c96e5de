// Reduction plans for the policies of Section 4 (see plan.hpp).
#include "plan.hpp"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <unordered_map>

namespace crf {

bool greedy_direction(const Family &fam, const int *U, int *v) {
    // Algorithm 3: one unit on every variable of S that U uses, then round
    // robin over all variables while v_i < U_i, until |v| = d.
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
        if (!moved) return false;
    }
    return true;
}

int direction_index(const Family &fam, const int *v) {
    for (int t = 0; t < fam.dirs.count; t++) {
        const int8_t *e = fam.dirs.at(t);
        bool eq = true;
        for (int i = 0; i < fam.nv; i++) eq = eq && e[i] == v[i];
        if (eq) return t;
    }
    return -1;
}

bool direction_valid(const Family &fam, const int *U, const int *v, int k) {
    for (int i = 0; i < fam.nv; i++) {
        if (U[i] - k * v[i] < 0) return false;
        if (((fam.smask >> i) & 1u) && v[i] == 0 && U[i] != 0) return false;
    }
    return true;
}

namespace {

// Algorithm 3 chunks from (U, pole) until pole == stop or, with var >= 0,
// U[var] == 0.  The chunk length is the largest k with U - k v >= 0, capped
// by the poles left.  Returns the pole reached (-1 if no direction exists).
int greedy_run(const Family &fam, int *U, int pole, int stop, int var, int64_t &chunks) {
    int v[kMaxVars];
    while (pole > stop) {
        if (var >= 0 && U[var] == 0) break;
        if (!greedy_direction(fam, U, v)) return -1;
        int k = pole - stop;
        for (int i = 0; i < fam.nv; i++)
            if (v[i]) k = std::min(k, U[i] / v[i]);
        if (k < 1) return -1;
        for (int i = 0; i < fam.nv; i++) U[i] -= k * v[i];
        pole -= k;
        chunks++;
    }
    return pole;
}

u64 coef_at(const ItemSetup &it, int crow, int col) {
    const int nch = it.nchain();
    if (crow < nch) return it.coef[(size_t)crow * it.b + col];
    return (crow - nch == col) ? 1 : 0;
}

struct UKey {
    int16_t u[kMaxVars];
    int nv;
    bool operator==(const UKey &o) const { return std::memcmp(u, o.u, sizeof(int16_t) * nv) == 0; }
};
struct UKeyHash {
    size_t operator()(const UKey &k) const {
        size_t h = 1469598103934665603ull;
        for (int i = 0; i < k.nv; i++) h = (h ^ (uint16_t)k.u[i]) * 1099511628211ull;
        return h;
    }
};

}  // namespace

namespace {

void init_terms(const Family &fam, const ItemSetup &it, std::vector<PlanTerm> &terms) {
    const int nv = fam.nv, b = it.b, nch = it.nchain();
    terms.assign(nch, PlanTerm{});
    for (int k = 0; k < nch; k++) {
        PlanTerm &t = terms[k];
        std::memset(t.u, 0, sizeof(t.u));
        for (int i = 0; i < nv; i++) t.u[i] = it.chain_u[(size_t)k * nv + i];
        t.pole = it.chain_pole[k];
        t.src = -(it.chain_g[k] + 1);
        t.crow = k;
        t.cols = 0;
        if (b <= 64)
            for (int c = 0; c < b; c++)
                if (it.coef[(size_t)k * b + c]) t.cols |= 1ull << c;
    }
}

// Reduces terms[active[a]] to stops[a] (Algorithm 3 chunks, ending early when
// u[var] reaches 0 if var >= 0; or the forced direction dirs[a] >= 0 for the
// whole range) and appends the phase's vectors to the plan.
bool run_phase(const Family &fam, ItemPlan &plan, std::vector<PlanTerm> &terms, const std::vector<int> &active,
               const std::vector<int> &stops, int var, const std::vector<int32_t> *forced, std::string &err,
               bool simulate = true) {
    const int nv = fam.nv, n = fam.n;
    std::vector<PlanVec> vecs;
    for (size_t a = 0; a < active.size(); a++) {
        PlanTerm &t = terms[active[a]];
        int U[kMaxVars] = {0};
        for (int i = 0; i < nv; i++) U[i] = t.u[i];
        PlanVec pv{};
        std::memcpy(pv.u, t.u, sizeof(pv.u));
        pv.pole = t.pole;
        pv.in = t.src >= 0 ? t.src : -1;
        pv.gamma = t.src < 0 ? -t.src - 1 : -1;
        pv.crow = t.crow;
        pv.dir = -1;
        int reached;
        const int fd = forced ? (*forced)[a] : -1;
        if (fd >= 0) {
            int v[kMaxVars] = {0};
            const int8_t *e = fam.dirs.at(fd);
            for (int i = 0; i < nv; i++) v[i] = e[i];
            const int k = t.pole - stops[a];
            if (k < 1 || !direction_valid(fam, U, v, k)) {
                err = "learned policy chose an invalid direction";
                return false;
            }
            for (int i = 0; i < nv; i++) U[i] -= k * v[i];
            reached = stops[a];
            plan.chunks++;
            pv.dir = fd;
        } else if (simulate || var >= 0) {
            reached = greedy_run(fam, U, t.pole, stops[a], var, plan.chunks);
        } else {
            reached = stops[a];  // Algorithm 3 runs on the device
        }
        if (reached < 0) {
            err = "no valid reduction direction (Algorithm 3)";
            return false;
        }
        if (reached == t.pole) continue;  // nothing to do in this phase
        pv.pend = reached;
        plan.column_steps += t.pole - reached;
        plan.vectors++;
        if (reached == n) {
            pv.out = -1;
            t.pole = -1;  // retired
        } else {
            pv.out = plan.nrows++;
            for (int i = 0; i < nv; i++) t.u[i] = (int16_t)U[i];
            t.pole = reached;
            t.src = pv.out;
        }
        vecs.push_back(pv);
    }
    std::stable_sort(vecs.begin(), vecs.end(),
                     [](const PlanVec &x, const PlanVec &y) { return x.pole - x.pend > y.pole - y.pend; });
    plan.phase.push_back(std::move(vecs));
    return true;
}

// Combines like terms among the live terms; the rows built here are read by the next phase.
void combine_terms(const Family &fam, const ItemSetup &it, ItemPlan &plan, std::vector<PlanTerm> &terms) {
    const int nv = fam.nv, n = fam.n, b = it.b, nch = it.nchain();
    std::vector<PlanComb> cb;
    std::unordered_map<UKey, std::vector<int>, UKeyHash> groups;
    for (int k = 0; k < (int)terms.size(); k++) {
        if (terms[k].pole <= n) continue;
        UKey key;
        std::memcpy(key.u, terms[k].u, sizeof(key.u));
        key.nv = nv;
        groups[key].push_back(k);
    }
    // deterministic order of the new rows: by the first member of each group
    std::vector<std::vector<int>> glist;
    for (auto &g : groups) glist.push_back(g.second);
    std::sort(glist.begin(), glist.end(), [](const std::vector<int> &x, const std::vector<int> &y) { return x[0] < y[0]; });
    std::vector<PlanTerm> next;
    std::vector<char> gone(terms.size(), 0);
    for (const std::vector<int> &mem : glist) {
        uint64_t cols = 0;
        for (int k : mem) cols |= terms[k].cols;
        const int na = __builtin_popcountll(cols);
        if ((int)mem.size() <= na) continue;
        plan.combined_groups++;
        plan.merged_terms += (int64_t)mem.size();
        for (int c = 0; c < b; c++) {
            if (!((cols >> c) & 1ull)) continue;
            PlanComb pc{plan.nrows++, (int32_t)plan.msrc.size(), 0};
            for (int k : mem) {
                const u64 a = coef_at(it, terms[k].crow, c);
                if (!a) continue;
                plan.msrc.push_back(terms[k].src);
                plan.malpha.push_back(a);
            }
            pc.m1 = (int32_t)plan.msrc.size();
            cb.push_back(pc);
            PlanTerm t = terms[mem[0]];
            t.src = pc.row;
            t.crow = nch + c;
            t.cols = 1ull << c;
            next.push_back(t);
        }
        for (int k : mem) gone[k] = 1;
    }
    std::vector<PlanTerm> kept;
    for (size_t k = 0; k < terms.size(); k++)
        if (!gone[k] && terms[k].pole > n) kept.push_back(terms[k]);
    for (auto &t : next) kept.push_back(t);
    terms.swap(kept);
    plan.comb.push_back(std::move(cb));
}

bool any_live(const std::vector<PlanTerm> &terms, int n) {
    for (auto &t : terms)
        if (t.pole > n) return true;
    return false;
}

}  // namespace

// ------------------------------------------------------------------ p-chunk phases
bool PChunkPlanner::init(const Family &f, const ItemSetup &s, int policy, std::string &err) {
    fam = &f;
    it = &s;
    plan = ItemPlan();
    plan.policy = policy;
    if (s.b > 64) {
        err = "combining policies need at most 64 basis columns";
        return false;
    }
    init_terms(f, s, terms);
    plan.comb.push_back({});
    started = finished = false;
    return true;
}

bool PChunkPlanner::begin_phase() {
    // Section 4.1: the terms of largest pole L are reduced to max(L - p, n)
    act.clear();
    int L = -1;
    for (auto &t : terms) L = std::max(L, t.pole);
    if (L <= fam->n) {
        finished = true;
        return false;
    }
    stop = std::max(L - it->p, fam->n);
    for (int k = 0; k < (int)terms.size(); k++)
        if (terms[k].pole > stop) act.push_back(k);
    started = true;
    return true;
}

void PChunkPlanner::candidates(std::vector<CandRow> &rows) const {
    const int nv = fam->nv, n = fam->n, d = fam->d, p = it->p;
    // landing of every active term under Algorithm 3 chunks, and the terms waiting at the stop pole:
    // for every landing exponent the list of (active index or -1, active columns)
    std::unordered_map<UKey, std::vector<std::pair<int, uint64_t>>, UKeyHash> land;
    for (size_t a = 0; a < act.size(); a++) {
        const PlanTerm &t = terms[act[a]];
        int U[kMaxVars] = {0};
        for (int i = 0; i < nv; i++) U[i] = t.u[i];
        int64_t dummy = 0;
        greedy_run(*fam, U, t.pole, stop, -1, dummy);
        UKey key;
        std::memset(key.u, 0, sizeof(key.u));
        for (int i = 0; i < nv; i++) key.u[i] = (int16_t)U[i];
        key.nv = nv;
        land[key].push_back({(int)a, t.cols});
    }
    for (const PlanTerm &t : terms) {
        if (t.pole != stop || stop <= n) continue;
        UKey key;
        std::memcpy(key.u, t.u, sizeof(key.u));
        key.nv = nv;
        land[key].push_back({-1, t.cols});
    }
    const float rem = (float)(stop - n) / (float)(p * (n + 1));
    for (size_t a = 0; a < act.size(); a++) {
        const PlanTerm &t = terms[act[a]];
        const int k = t.pole - stop;
        int U[kMaxVars] = {0}, g[kMaxVars] = {0};
        int un = 0;
        for (int i = 0; i < nv; i++) {
            U[i] = t.u[i];
            un += U[i];
        }
        const bool has_greedy = greedy_direction(*fam, U, g);
        for (int di = 0; di < fam->dirs.count; di++) {
            const int8_t *e = fam->dirs.at(di);
            int v[kMaxVars] = {0};
            for (int i = 0; i < nv; i++) v[i] = e[i];
            if (!direction_valid(*fam, U, v, k)) continue;
            CandRow r{};
            r.term = (int32_t)a;
            r.dir = di;
            UKey key;
            std::memset(key.u, 0, sizeof(key.u));
            bool same_greedy = has_greedy;
            for (int i = 0; i < nv; i++) {
                key.u[i] = (int16_t)(U[i] - k * v[i]);
                same_greedy = same_greedy && g[i] == v[i];
            }
            key.nv = nv;
            int cnt = 0;  // the other terms there (the plain plan may already have put this one there)
            uint64_t cols = 0;
            auto f = land.find(key);
            if (f != land.end())
                for (const auto &mem : f->second)
                    if (mem.first != (int)a) {
                        cnt++;
                        cols |= mem.second;
                    }
            for (int i = 0; i < nv; i++) {
                r.x[i] = un ? (float)U[i] / (float)un : 0.f;
                r.x[6 + i] = (float)v[i] / (float)d;
            }
            r.x[12] = std::log1p((float)__builtin_popcountll(cols)) / 4.f;
            r.x[13] = rem;
            r.x[14] = std::log1p((float)cnt) / 4.f;
            r.x[15] = same_greedy ? 1.f : 0.f;
            const int before = std::min(cnt, __builtin_popcountll(cols));
            const int after = std::min(cnt + 1, __builtin_popcountll(cols | t.cols));
            r.label = (float)(after - before) * rem;
            rows.push_back(r);
        }
    }
}

bool PChunkPlanner::end_phase(const std::vector<int32_t> &dir, std::string &err) {
    std::vector<int> stops(act.size(), stop);
    const bool any_forced = std::any_of(dir.begin(), dir.end(), [](int32_t x) { return x >= 0; });
    if (!run_phase(*fam, plan, terms, act, stops, -1, any_forced ? &dir : nullptr, err)) return false;
    if (any_live(terms, fam->n)) combine_terms(*fam, *it, plan, terms);
    return true;
}

int64_t depth_first_chunks(const Family &fam, const ItemSetup &it) {
    int64_t chunks = 0;
    for (int k = 0; k < it.nchain(); k++) {
        int U[kMaxVars] = {0};
        for (int i = 0; i < fam.nv; i++) U[i] = it.chain_u[(size_t)k * fam.nv + i];
        if (greedy_run(fam, U, it.chain_pole[k], fam.n, -1, chunks) != fam.n) return -1;
    }
    return chunks;
}

bool plan_item(const Family &fam, const ItemSetup &it, int policy, ItemPlan &plan, std::string &err,
               bool count_chunks) {
    const int nv = fam.nv, n = fam.n, nch = it.nchain();
    if (policy == CR_POLICY_P_CHUNK) {
        PChunkPlanner pc;
        if (!pc.init(fam, it, policy, err)) return false;
        while (pc.begin_phase()) {
            std::vector<int32_t> none(pc.act.size(), -1);
            if (!pc.end_phase(none, err)) return false;
        }
        plan = std::move(pc.plan);
        return true;
    }
    plan = ItemPlan();
    plan.policy = policy;
    std::vector<PlanTerm> terms;
    init_terms(fam, it, terms);
    plan.comb.push_back({});
    if (policy == CR_POLICY_DEPTH_FIRST) {
        std::vector<int> act(nch), stops(nch, n);
        for (int k = 0; k < nch; k++) act[k] = k;
        return run_phase(fam, plan, terms, act, stops, -1, nullptr, err, count_chunks);
    }
    if (policy == CR_POLICY_VAR_BY_VAR) {
        if (it.b > 64) {
            err = "combining policies need at most 64 basis columns";
            return false;
        }
        // Section 4.3: reduce every term until its last variable vanishes, combine,
        // then the next variable; whatever is left goes to pole n
        for (int var = nv - 1; var >= -1; var--) {
            std::vector<int> act, stops;
            for (int k = 0; k < (int)terms.size(); k++)
                if (terms[k].pole > n && (var < 0 || terms[k].u[var] != 0)) {
                    act.push_back(k);
                    stops.push_back(n);
                }
            if (act.empty()) continue;
            if (!run_phase(fam, plan, terms, act, stops, var, nullptr, err)) return false;
            if (!any_live(terms, n)) break;
            combine_terms(fam, it, plan, terms);
        }
        return true;
    }
    if (policy == CR_POLICY_LEARNED) {
        err = "the learned policy is planned batch-wise with its network";
        return false;
    }
    err = "unknown policy";
    return false;
}

}  // namespace crf
