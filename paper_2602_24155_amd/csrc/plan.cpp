// Reduction plans for the policies of Section 4 (see plan.hpp).
#include "plan.hpp"

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

bool plan_item(const Family &fam, const ItemSetup &it, int policy, ItemPlan &plan, std::string &err,
               const DirChooser *chooser) {
    const int nv = fam.nv, n = fam.n, b = it.b, nch = it.nchain();
    plan = ItemPlan();
    plan.policy = policy;
    std::vector<PlanTerm> terms(nch);
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
    if (policy != CR_POLICY_DEPTH_FIRST && b > 64) {
        err = "combining policies need at most 64 basis columns";
        return false;
    }
    if (policy == CR_POLICY_LEARNED && !chooser) {
        err = "learned policy without a direction chooser";
        return false;
    }

    // reduce the terms selected by `active` of one phase; stop pole per term from stop_of
    auto run_phase = [&](const std::vector<int> &active, const std::vector<int> &stops, int var,
                         const std::vector<int32_t> *forced) -> bool {
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
            } else {
                reached = greedy_run(fam, U, t.pole, stops[a], var, plan.chunks);
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
    };

    // combine like terms among the live terms; the rows built here are read by the next phase
    auto combine = [&]() {
        std::vector<PlanComb> cb;
        std::unordered_map<UKey, std::vector<int>, UKeyHash> groups;
        for (int k = 0; k < (int)terms.size(); k++) {
            if (terms[k].pole <= n) continue;
            UKey key;
            std::memcpy(key.u, terms[k].u, sizeof(key.u));
            key.nv = nv;
            groups[key].push_back(k);
        }
        std::vector<PlanTerm> next;
        std::vector<char> gone(terms.size(), 0);
        for (auto &g : groups) {
            const std::vector<int> &mem = g.second;
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
    };

    plan.comb.push_back({});
    if (policy == CR_POLICY_DEPTH_FIRST) {
        std::vector<int> act(nch), stops(nch, n);
        for (int k = 0; k < nch; k++) act[k] = k;
        if (!run_phase(act, stops, -1, nullptr)) return false;
        return true;
    }
    if (policy == CR_POLICY_VAR_BY_VAR) {
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
            if (!run_phase(act, stops, var, nullptr)) return false;
            bool live = false;
            for (auto &t : terms) live = live || t.pole > n;
            if (!live) break;
            combine();
        }
        return true;
    }
    if (policy == CR_POLICY_P_CHUNK || policy == CR_POLICY_LEARNED) {
        // Section 4.1: the terms of largest pole L are reduced to max(L - p, n), like
        // terms are combined, and so on (start poles are multiples of p)
        for (;;) {
            int L = -1;
            for (auto &t : terms) L = std::max(L, t.pole);
            if (L <= n) break;
            const int stop = std::max(L - it.p, n);
            std::vector<int> act, stops;
            std::vector<PlanTerm> sel;
            for (int k = 0; k < (int)terms.size(); k++)
                if (terms[k].pole > stop) {
                    act.push_back(k);
                    stops.push_back(stop);
                    sel.push_back(terms[k]);
                }
            std::vector<int32_t> forced;
            if (policy == CR_POLICY_LEARNED) {
                if (!(*chooser)(sel, stop, forced) || forced.size() != sel.size()) {
                    err = "learned policy failed to choose directions";
                    return false;
                }
            }
            if (!run_phase(act, stops, -1, policy == CR_POLICY_LEARNED ? &forced : nullptr)) return false;
            bool live = false;
            for (auto &t : terms) live = live || t.pole > n;
            if (!live) break;
            combine();
        }
        return true;
    }
    err = "unknown policy";
    return false;
}

}  // namespace crf
