// Reduction plans: which start terms are reduced together, in which order,
// and where like terms are combined (Section 3.4's reduction game, the
// policies of Section 4).
//
// A plan is a list of phases.  In a phase every active term is reduced as one
// vector from its pole to the phase's stop pole; between phases, terms whose
// exponents u coincide (and hence whose poles coincide) may be combined.  The
// value of a term is always  w (x) c : a vector w over Homog_{dn-n} times a row
// c of coefficients over the basis columns.  Start terms are rank one (w a unit
// vector e_gamma, c the Proposition 2.1 coefficients of their x^S-form
// exponent); combining a group of terms with active columns A replaces them by
// |A| vectors w_a = sum_j c_j[a] w_j with unit rows e_a.  A group is combined
// only when it holds more vectors than active columns, so combining never
// increases the number of vectors that are reduced.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "host.hpp"

namespace crf {

// One vector of a phase.  It starts at exponent u and pole `pole` from the
// unit vector e_gamma (in < 0) or from store row `in`, is reduced to pole
// `pend`, and ends in store row `out` (read by a later combine or phase) or,
// when out < 0 (then pend = n), in the pole-n numerators of the final
// Griffiths-Dwork step.  dir >= 0 forces one direction for the whole range
// (pole - pend steps, valid by construction); dir < 0 reduces by Algorithm 3
// chunks capped at pend.
struct PlanVec {
    int16_t u[kMaxVars];
    int32_t pole, pend, gamma, in, out, dir;
    int32_t crow;  // coefficient row used by the final assembly (see ItemPlan)
};

// A store row built between two phases: row = sum_{j in [m0, m1)} alpha_j src_j,
// src_j >= 0 a store row, src_j < 0 the unit vector e_{-src_j - 1}.
struct PlanComb {
    int32_t row, m0, m1;
};

struct ItemPlan {
    int policy = 0;
    std::vector<std::vector<PlanVec>> phase;  // phase t, each sorted by steps (pole - pend) descending
    std::vector<std::vector<PlanComb>> comb;  // comb[t]: rows built before phase t (comb[0] empty)
    std::vector<int32_t> msrc;                // members of every PlanComb
    std::vector<u64> malpha;
    int32_t nrows = 0;                        // store rows (s residues each)
    // coefficient rows: crow < nchain is start row crow of ItemSetup::coef,
    // crow >= nchain the unit row of basis column crow - nchain
    int64_t column_steps = 0, chunks = 0, vectors = 0, merged_terms = 0, combined_groups = 0;
};

// A term of the reduction game as the planner sees it.
struct PlanTerm {
    int16_t u[kMaxVars];
    int32_t pole;
    int32_t src;   // store row, or -(gamma + 1) for a unit start vector
    int32_t crow;
    uint64_t cols; // active basis columns
};

// Inputs of the learned policy's scoring network, one row per (term,
// candidate direction) of a p-chunk phase.  For a term at exponent u reduced
// by k = pole - stop steps with direction v to u' = u - k v:
//   x[0..5]  u_i / |u|            x[6..11] v_i / d
//   x[12]    log(1 + |A|) / 4     x[13]    (stop - n) / (p (n + 1))
//   x[14]    log(1 + g) / 4, g = terms landing at u' in the plain p-chunk plan
//            (other than this term) plus terms already waiting at u'; A = the
//            active basis columns of those terms
//   x[15]    1 if v is Algorithm 3's direction for u
// label = the vectors this choice adds at u' (min(g + 1, |A + A_t|) -
// min(g, |A|), A the active columns there, A_t the term's) times
// (stop - n) / (p (n + 1)): the remaining work it causes.
constexpr int kMlpIn = 16;
struct CandRow {
    int32_t term, dir;
    float x[kMlpIn];
    float label;
};

// The p-chunk phases of one item as a state machine, so that the directions
// of a whole batch can be chosen phase by phase (one network evaluation per
// phase for every item).
struct PChunkPlanner {
    const Family *fam = nullptr;
    const ItemSetup *it = nullptr;
    ItemPlan plan;
    std::vector<PlanTerm> terms;
    std::vector<int> act;  // terms of the current phase
    int stop = 0;
    bool started = false, finished = false;
    bool init(const Family &f, const ItemSetup &s, int policy, std::string &err);
    // Selects the next phase; false when every term has reached pole n.
    bool begin_phase();
    // Candidate rows of the current phase (features and labels).
    void candidates(std::vector<CandRow> &rows) const;
    // Reduces the phase with dir[a] for act[a] (-1: Algorithm 3 chunks), then combines.
    bool end_phase(const std::vector<int32_t> &dir, std::string &err);
};

// Game cost used to judge a plan (Section 3.4 with M = 1 per column step,
// S = 0 per chunk: no matrix is materialised per chunk here, and D = 1/8 per
// merged term: a combine reads one vector instead of an s x s product).
inline double plan_cost(const ItemPlan &p) { return (double)p.column_steps + 0.125 * (double)p.merged_terms; }

// Algorithm 3 for exponent U (greedy v); false if no direction exists.
bool greedy_direction(const Family &fam, const int *U, int *v);
// Index of direction v among fam.dirs, or -1.
int direction_index(const Family &fam, const int *v);
// Whether direction v can be used for k consecutive steps from exponent U:
// U - k v >= 0, and i in S with v_i = 0 implies U_i = 0.
bool direction_valid(const Family &fam, const int *U, const int *v, int k);

// Builds the plan of one item for a plain policy (depth-first, p-chunk,
// var-by-var).  Requires b <= 64 for the combining policies.  With
// count_chunks false, the depth-first plan does not run Algorithm 3 along
// every chain (the device chooses the directions itself): plan.chunks stays 0
// and depth_first_chunks() gives it later.
bool plan_item(const Family &fam, const ItemSetup &it, int policy, ItemPlan &plan, std::string &err,
               bool count_chunks = true);
// Algorithm 3 chunks of the depth-first reduction of every start vector of
// the item to pole n; -1 if some vector has no valid direction.
int64_t depth_first_chunks(const Family &fam, const ItemSetup &it);

}  // namespace crf
