/*
 * crfrob -- controlled reduction of hypersurface zeta functions on AMD MI355X.
 *
 * C ABI of libcrfrob.so.  Plain pointers and sizes only; every call returns a
 * cr_status (0 = CR_OK) and never throws.  On error the outputs of the failing
 * item are left untouched and cr_last_error() describes the failure.
 *
 * Mathematics (arXiv 2602.24155): X = V(f) a smooth hypersurface of degree d
 * in P^n over F_p, 7 <= p < 50.  Its zeta function is
 *   Z(X,T) = Q(T)^((-1)^n) / prod_{i<n} (1 - p^i T)            (Section 2.1)
 * with Q(T) = det(1 - T Phi), Phi the matrix of p^{-1} sigma on H^n_dR(U) in
 * the monomial basis of Section 2.3.  The library returns the matrix Phi'
 * whose column c holds the coordinates of p^(m_c - n - 1) sigma(x^beta Omega
 * / f^m_c) (Proposition 2.1), so Phi = Phi' diag(p^(n - m_c)), and the
 * integer coefficients of Q(T).
 *
 * Conventions shared by every entry point:
 *  - nvars = n + 1 variables, 3 <= nvars <= 6; degree d >= 2.
 *  - Coefficients are listed in lexicographically DESCENDING order of the
 *    exponent vectors of the degree-d monomials (x_0^d first; cr_monomials
 *    returns that list) and are the representatives in [0, p) of the F_p
 *    coefficients; this integer polynomial is the lift f of Section 2.1.
 *  - Basis of H^n_dR(U): for m = 1..n the degree dm-n-1 monomials that are
 *    not pivot columns of the row-echelon form (mod p) of the image of
 *    (mu_i) -> sum mu_i d_i f, monomials scanned in the order above
 *    (Section 2.3).  Basis elements are ordered by m, then by that order.
 *  - Precision (Section 2.5): one relative precision r for all columns, the
 *    smallest that recovers every a_i (i <= b/2) of Q(T) from the Weil bound
 *    either directly (a_i mod p^(r + h_i)) or through the power sum
 *    tr(Phi^i); series order N_m = r + 1; working modulus p^M with
 *    M = max_m (r + v_p((p s_m - 1)!) - m + 1), s_m = N_m + m - 1.
 *  - The Frobenius series coefficients D_{j,m} C_{j,alpha} of Proposition 2.1
 *    are taken exactly and reduced mod p^M.
 */
#ifndef CRFROB_H
#define CRFROB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CR_OK = 0,
    CR_EINVAL = 1,        /* bad sizes / null pointers / unsupported nvars, degree, or a family
                             with no device path (a right inverse beyond 2^20 entries and no
                             MFMA kernel: cubic fourfolds) */
    CR_ENOTPRIME = 2,     /* p is not prime */
    CR_EPRANGE = 3,       /* need 7 <= p < 50, p > n, p not dividing d */
    CR_ESINGULAR = 4,     /* f mod p is singular (Jacobian criterion) */
    CR_ENOT_S_SMOOTH = 5, /* f is smooth but not S-smooth for the requested S (Definition 3.1) */
    CR_EPRECISION = 6,    /* p^M does not fit the 64-bit residues of this build */
    CR_ENOMEM = 7,        /* host or device allocation failed */
    CR_EDEVICE = 8,       /* HIP runtime error, or no gfx950 device */
    CR_ESELFCHECK = 9     /* a built-in consistency check failed (divisibility of a
                             column, det Phi' = +-1 mod p, integrality of Newton's identities) */
} cr_status;

/* Reduction policies (Section 4).  Every policy yields the same Phi' bits:
 * each reduction step is an exact identity in cohomology and the
 * coordinates of a class are unique. */
typedef enum {
    CR_POLICY_DEPTH_FIRST = 0, /* Section 4.2: per term greedy v (Algorithm 3), largest chunk k
                                  with v in V_full(u, k); never combines like terms */
    CR_POLICY_P_CHUNK = 1,     /* Section 4.1: the terms of largest pole L are reduced to
                                  max(L - p, n) by Algorithm 3 chunks, then like terms (equal
                                  exponent u) are combined; repeat */
    CR_POLICY_VAR_BY_VAR = 2,  /* Section 4.3: reduce every term until u_n = 0, combine, then
                                  u_{n-1}, ..., u_0; the rest goes to pole n */
    CR_POLICY_LEARNED = 3      /* the p-chunk phases with each term's direction chosen by a
                                  trained MLP (cr_mlp_*), judged against the plain policies by
                                  the game cost of Section 3.4 (falls back when it loses) */
} cr_policy;

/* Combining like terms (Section 3.4, second move of the game): a term is a
 * vector w over Homog_{dn-n} times a row c of basis-column coefficients.  A
 * group of terms with equal exponent u and active columns A is replaced by
 * |A| vectors sum_j c_j[a] w_j (one per column a in A) when it holds more
 * than |A| terms; smaller groups are left as they are. */

/* Learned policy model (opaque): a fully connected fp32 network 16 -> 128 ->
 * 128 -> 1 (ReLU) that scores (term, candidate direction) pairs of a p-chunk
 * phase; see cr_mlp_create. */
typedef struct cr_mlp cr_mlp;

/* A family of hypersurfaces that share nvars, degree and S; p may vary per item. */
typedef struct {
    int32_t nvars;    /* n + 1 */
    int32_t degree;   /* d */
    uint32_t s_mask;  /* S of Definition 3.1 as a bit set over x_0..x_n; 0 = all variables */
    int32_t policy;   /* cr_policy */
    int32_t r;        /* relative precision override; 0 = derive (header comment) */
    int32_t n_series; /* series order override N_m for every m; 0 = r + 1 */
    int32_t engine;   /* reduction kernel: 0 = auto (int8-digit MFMA kernel with the gather on
                         the accumulators and two interleaved tiles per workgroup -- the
                         products of one tile overlap the finishing of the other -- for the
                         items whose digit count allows it (5 or 8 digits for plane quintics),
                         the same kernel with one tile per workgroup for the other items of the
                         batch (10 digits), for four-variable families with S = all (quartic K3
                         surfaces) the quad kernel, for cubic threefolds with S = {x_4} and
                         quintic surfaces the streaming kernel, else the 64-bit VALU
                         kernel), 1 = 64-bit VALU
                         kernel, 2 = int8-digit MFMA kernel with the gather through LDS, 3 =
                         register-gather MFMA kernel with one tile per workgroup, 4 = quad
                         kernel: int8-digit MFMA for four variables, psi digits streamed from
                         memory row tile by row tile, the gather on the accumulators (each
                         output's source rows in one lane's aligned quad of rows), 5 =
                         streaming kernel: the same for cubic threefolds with S = {x_4} (57
                         row tiles, 32 K-blocks, each output's five source rows in one
                         lane) and quintic surfaces (28 row tiles, 18 K-blocks, the quad
                         placement), the vectors' digit planes in global memory, always
                         in its persistent form */
    int32_t launch;   /* reduction launches (int8-digit register-gather and quad kernels; the
                         others always use mode 0): 0 = one workgroup per tile of 32 vectors; 1 = persistent:
                         one grid sized to the device's resident capacity drains the tiles
                         (longest first) through an atomic counter; 2 = as 1, with the launches
                         of a sub-batch captured once into a hipGraph and replayed while the
                         launch parameters repeat */
    cr_mlp *mlp;      /* model of CR_POLICY_LEARNED (required then, ignored otherwise); the
                         library uses its device scratch, so one model serves one call at a time */
    int32_t M;        /* working precision override (Section 2.5: the modulus p^M of the
                         reduction); 0 = the least M that keeps r digits in every column (header
                         comment).  A smaller M is rejected (CR_EINVAL); a larger one computes
                         more digits of every column (col_prec grows by the difference) */
    int32_t n_series_m[6]; /* per pole order override of N_m (Proposition 2.1: the Frobenius
                         series of a column of pole m is truncated after N_m terms), entry m-1
                         for m = 1..n; 0 = n_series (or r + 1) */
    int32_t grid;     /* persistent launches (launch >= 1): workgroups per CU of the grid, 1..4;
                         0 = 1 */
} cr_family;

/* Per-call statistics (all counts are summed over the batch). */
typedef struct {
    int64_t start_blocks;    /* distinct Frobenius start terms (x^S form exponents) */
    int64_t column_steps;    /* s x s . s reduction products (the paper's unit M of Section 3.4) */
    int64_t chunks;          /* reduction chunks (u, v, k): the startup cost S of Section 3.4 */
    int64_t vectors;         /* vectors reduced (start terms and combined columns, every phase) */
    int64_t merged_terms;    /* terms absorbed by combining like terms (cost D each) */
    int64_t combined_groups; /* groups of like terms that were combined */
    double setup_ms;         /* host setup and planning wall time */
    double device_ms;        /* device time of the reduction, combine and assembly kernels */
    double reduce_ms;        /* device time of the reduction kernels (HIP events) */
    double combine_ms;       /* device time of the combine kernels */
    double assemble_ms;      /* device time of the Griffiths-Dwork assembly kernel */
    double finish_ms;        /* host unscaling and L-polynomial recovery */
    int32_t engine;          /* kernel that ran: 0 / 3 / 2 = int8-digit MFMA (register gather with tile
                                pairs for some or all items / with one tile / LDS gather), 4 = int8-digit MFMA quad kernel
                                (four variables), 5 = int8-digit MFMA streaming kernel (cubic threefolds,
                                quintic surfaces), 1 = 64-bit VALU */
    int32_t policy;          /* policy whose plan ran */
    int32_t phases;          /* reduction phases (combine points + 1) of the longest plan */
    int32_t fallbacks;       /* CR_POLICY_LEARNED: items whose learned plan cost more than a
                                plain policy's and were reduced with the cheaper plain plan */
    int64_t reduce_launches; /* launches of the reduction kernels (sub-batches x phases x digit groups) */
    double psi_ms;           /* device time of the right inverses of J_S (one launch per call, every item) */
} cr_stats;

/* Sizes: ncoeff = C(d+n, n); s = C(dn, n) = dim Homog_{dn-n} (side of R_{u,v},
 * Proposition 3.3); b = dimension of H^n_dR(U) (side of Phi', the sum over
 * m = 1..n of the basis sizes of Section 2.3).  Pure function of (nvars,
 * degree); outputs may be NULL.  CR_EINVAL for unsupported nvars / degree. */
cr_status cr_query_dims(int32_t nvars, int32_t degree, int32_t *ncoeff, int32_t *s, int32_t *b);

/* Section 2.1 (the lift of f): the exponent vectors of the degree-d monomials
 * in the order in which every entry point takes the coefficients of f,
 * lexicographically descending: exps[k * nvars + i] = exponent of x_i in
 * monomial k.  exps is caller-owned, ncoeff * nvars entries.  CR_EINVAL for a
 * null pointer or unsupported nvars / degree. */
cr_status cr_monomials(int32_t nvars, int32_t degree, int32_t *exps);

/* Section 2.5: precision chosen for prime p under fam's overrides (header
 * comment): the relative precision r, the largest series order N_m over
 * m = 1..n (all equal unless fam->n_series_m sets some) and the working
 * precision M.  Outputs may be NULL.  CR_EINVAL if an override is out of
 * range or fam->M is below the least working precision. */
cr_status cr_precision(const cr_family *fam, int32_t p, int32_t *r, int32_t *n_series, int32_t *M);

/* Words per residue of the Frobenius outputs for prime p (Section 2.5: the
 * coordinates are residues mod p^M): 1 when p^M < 2^55, the residues of this
 * build.  Larger moduli are rejected here and by every computing entry point
 * with CR_EPRECISION.  Host only. */
cr_status cr_residue_words(const cr_family *fam, int32_t p, int32_t *words);

/* Definition 3.1: *smooth = 1 iff f mod p is smooth (Jacobian criterion) and,
 * for fam->s_mask != 0, S-smooth (J_S : (+)_{i in S} Homog_{D-d+1} (+)
 * (+)_{i not in S} Homog_{D-d} -> Homog_D surjective mod p); 0 otherwise.  The
 * status is CR_OK either way for valid arguments; CR_EINVAL for null
 * pointers or a bad family, CR_ENOTPRIME / CR_EPRANGE for p.  Host only. */
cr_status cr_check_smooth(const cr_family *fam, int32_t p, const uint32_t *coeffs, int32_t *smooth);

/*
 * Frobenius matrices and L-polynomials of `count` hypersurfaces of one family
 * (Sections 2-4): host setup (Section 2.3-2.5, Proposition 2.1, decomposition
 * map of Proposition 3.3, Griffiths-Dwork map of Section 3.3), one batched
 * device reduction of every start term to pole order n (Proposition 3.3 with
 * the explicit R_{u,v} of Section 3.1, Algorithm 2 order of evaluation), the
 * device Griffiths-Dwork assembly, host unscaling and Q(T).
 *
 *   primes     [count]            p of each item
 *   coeffs     [count * ncoeff]   coefficients in [0, p), cr_monomials order
 *   frob       [count * b * b]    Phi' residues, row-major; column c is known
 *                                 mod p^col_prec[c]
 *   frob_scaled[count * b * b]    may be NULL: the coordinates before unscaling,
 *                                 exact mod p^M (the quantity every reduction
 *                                 policy reproduces bit for bit)
 *   col_pole   [count * b]        pole order m of each column
 *   col_prec   [count * b]        p-adic digits known in each column of Phi'
 *   lpoly      [count * (b+1) * 4] Q(T) coefficients a_0..a_b, each a signed
 *                                 256-bit two's-complement integer as four
 *                                 little-endian uint64 words; a_0 = 1
 *   item_status[count]            per-item cr_status (may be NULL)
 *   stats      may be NULL
 *   hip_stream hipStream_t of the caller, or NULL for the default stream
 * All buffers are host memory owned by the caller.  Device memory is owned by
 * the library (kept across calls and reused) and freed by cr_release().
 * Returns CR_OK if every item succeeded, else the first failing item's status.
 */
cr_status cr_frobenius_batch(const cr_family *fam, int32_t count, const int32_t *primes,
                             const uint32_t *coeffs, uint64_t *frob, uint64_t *frob_scaled,
                             int32_t *col_pole, int32_t *col_prec, int64_t *lpoly,
                             int32_t *item_status, cr_stats *stats, void *hip_stream);

/* One hypersurface (the same path as cr_frobenius_batch with count = 1; its
 * buffers are those of one batch item): Sections 2-4 for f with coefficients
 * coeffs[ncoeff] at prime p.  frob[b * b], frob_scaled[b * b] (may be NULL),
 * col_pole[b], col_prec[b], lpoly[(b + 1) * 4] as in cr_frobenius_batch.
 * Returns the item's status. */
cr_status cr_frobenius(const cr_family *fam, int32_t p, const uint32_t *coeffs, uint64_t *frob, uint64_t *frob_scaled,
                       int32_t *col_pole, int32_t *col_prec, int64_t *lpoly, cr_stats *stats, void *hip_stream);

/* For callers that cannot allocate device memory (work inside their own HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, arguments, outputs and per-item statuses as
 * cr_frobenius_batch, with every device buffer taken from one static
 * workspace of CR_NOALLOC_WORKSPACE_BYTES bytes inside the library (each
 * device holds its own copy from the first call on it until the process
 * ends).  The call makes no hipMalloc / hipFree / hipHostMalloc and creates
 * no stream or graph: host staging is pageable memory and every copy and
 * kernel runs on hip_stream.  The call's right inverses of J_S take the
 * front of the workspace and each sub-batch in turn the rest (so the host's
 * preparation of a sub-batch does not overlap the device work of the one
 * before); when they do not fit, the call fails with CR_ENOMEM and
 * cr_last_error() gives the bytes needed and held (a sub-batch of 24 plane
 * quintics under p-chunk needs about 82 MB).
 * CR_POLICY_LEARNED and launch mode 2 are rejected (CR_EINVAL).  Every call
 * on a device uses the same workspace and leaves its contents behind; each
 * call clears what must start at zero and returns only after its device work
 * is done.  Calls of one process are serialised by the library's lock; two
 * calls that overlapped on one device would race on the workspace. */
#define CR_NOALLOC_WORKSPACE_BYTES (128ull << 20)
cr_status cr_frobenius_batch_noalloc(const cr_family *fam, int32_t count, const int32_t *primes,
                                     const uint32_t *coeffs, uint64_t *frob, uint64_t *frob_scaled, int32_t *col_pole,
                                     int32_t *col_prec, int64_t *lpoly, int32_t *item_status, cr_stats *stats,
                                     void *hip_stream);

/* Host-only planning of one hypersurface under fam->policy (no device work):
 * fills start_blocks, column_steps, chunks, vectors, merged_terms,
 * combined_groups, phases and policy of *stats (the game cost of Section 3.4
 * is M column_steps + S chunks + D merged_terms).  Not available for
 * CR_POLICY_LEARNED (whose plan needs the model): CR_EINVAL. */
cr_status cr_policy_cost(const cr_family *fam, int32_t p, const uint32_t *coeffs, cr_stats *stats);

/*
 * Learned policy (an extension of the method: the paper's Section 4.4 asks
 * for better policies).  The network's inputs for a term at exponent u of a
 * p-chunk phase that ends at pole `stop`, and a direction v valid for all
 * k = pole - stop steps (u' = u - k v):
 *   x[0..5]  u_i/|u| (zero padded)     x[6..11] v_i/d (zero padded)
 *   x[12]    log(1 + |A|)/4            x[13]    (stop - n)/(p (n + 1))
 *   x[14]    log(1 + g)/4, g = other terms that land on u' in the plain p-chunk
 *            plan or already wait there; A = their active basis columns
 *   x[15]    1 if v is Algorithm 3's direction for u, else 0
 * Training label: the vectors the choice adds at u' (min(g + 1, |A u A_t|) -
 * min(g, |A|), A the active basis columns there, A_t the term's) times
 * (stop - n)/(p (n + 1)).  The policy takes, for every term, the candidate of
 * lowest score (ties: lowest direction index; no candidate: Algorithm 3
 * chunks), then judges the plan by the game cost of Section 3.4 with M = 1,
 * S = 0, D = 1/8 against the depth-first and p-chunk plans and reduces with
 * the cheapest.  The policy changes which vectors are reduced, never the bits.
 *
 * Parameters (CR_MLP_PARAMS floats, row-major, W[k][j] takes input k to unit j):
 *   W1[16][128], b1[128], W2[128][128], b2[128], w3[128], b3.
 */
#define CR_MLP_INPUTS 16
#define CR_MLP_HIDDEN 128
#define CR_MLP_PARAMS 18817

typedef struct {
    int32_t epochs;    /* passes over the rows */
    int32_t batch;     /* rows per Adam step (>= 1) */
    float lr, beta1, beta2, eps;  /* Adam; zeros select 1e-3, 0.9, 0.999, 1e-8 */
    uint64_t seed;     /* row shuffling */
} cr_train_opts;

/* New model on the current HIP device.  weights: CR_MLP_PARAMS floats, or NULL
 * for a seeded initialisation (weights uniform in +-1/sqrt(fan_in), biases 0). */
cr_status cr_mlp_create(const float *weights, uint64_t seed, cr_mlp **out);
cr_status cr_mlp_destroy(cr_mlp *m);
/* Copies the CR_MLP_PARAMS parameters to host memory. */
cr_status cr_mlp_weights(const cr_mlp *m, float *out);
/* Scores of `rows` input rows (host x[rows * 16] -> host y[rows]), on the GPU. */
cr_status cr_mlp_forward(cr_mlp *m, int32_t rows, const float *x, float *y, void *hip_stream);
/* Gradient of the loss (1/rows) sum (y - t)^2 with respect to the parameters
 * (host grad[CR_MLP_PARAMS]) and the loss, on the GPU. */
cr_status cr_mlp_grad(cr_mlp *m, int32_t rows, const float *x, const float *t, float *grad, float *loss,
                      void *hip_stream);
/* Adam on the GPU over host rows (x[rows * 16], labels t[rows]); loss[epochs]
 * (may be NULL) receives the mean minibatch loss of each epoch. */
cr_status cr_mlp_train(cr_mlp *m, int32_t rows, const float *x, const float *t, const cr_train_opts *opts,
                       float *loss, void *hip_stream);
/* Training rows of one hypersurface: the inputs and labels of every (term,
 * candidate) pair of its plain p-chunk plan.  With x == NULL only *rows is
 * set (the count); otherwise at most cap rows are written (CR_EINVAL if the
 * count exceeds cap). Host only. */
cr_status cr_trace_policy(const cr_family *fam, int32_t p, const uint32_t *coeffs, int32_t cap, float *x, float *t,
                          int32_t *rows);

/* Autotuner of the batched launch (an extension of the method; the paper
 * parallelises only across CPU threads, Sections 5.1 and 7).  Stage 1 runs
 * the batch under every (policy, launch) pair -- policies depth-first,
 * p-chunk, var-by-var (and learned when fam->mlp is set), launch modes 0, 1,
 * 2 -- with fam's engine and grid; stage 2 runs the fastest pair under every
 * kernel shape the family supports: engine (tile pairs, single tiles, LDS
 * gather, quad, VALU) x persistent grid (1 or 2 workgroups per CU).  Each
 * configuration runs once to warm up and `trials` times timed (wall clock of
 * whole cr_frobenius_batch calls); configurations whose kernel differs from
 * the one requested (cr_stats.engine) are not counted, nor calls that fail,
 * except that items reporting CR_EPRECISION after a reduction that ran (an
 * overridden precision too small to recover Q(T); their Frobenius matrices
 * are still computed) count as done.  Every configuration gives the same
 * bits.
 *   ms[policy * 3 + launch]   stage-1 mean times (-1 when not run)
 *   shape_ms[k]               stage-2 mean times for the shapes
 *                             (engine, grid) = (0,1) (0,2) (3,1) (3,2) (2,1) (4,1) (4,2) (1,1)
 * When a cache file is set (cr_autotune_cache), a result for the same family,
 * batch (count and primes) and device is read from it instead of timing
 * (from_cache = 1), and new results are appended to it. */
typedef struct {
    int32_t best_policy, best_launch;
    double best_ms;
    double ms[12];
    int32_t best_engine, best_grid;
    int32_t from_cache;
    double shape_ms[8];
} cr_tuning;
cr_status cr_autotune(const cr_family *fam, int32_t count, const int32_t *primes, const uint32_t *coeffs,
                      int32_t trials, cr_tuning *out, void *hip_stream);
/* File of persisted autotuner results (one line per tuned batch), or NULL to
 * stop using one.  The path is copied. */
cr_status cr_autotune_cache(const char *path);

/*
 * Newton-polygon invariants of Q(T) (host only; Sections 1.2, 6.3, 6.4, 6.6).
 * The Newton polygon is the lower convex hull of the points (j, v_p(a_j)) of
 * the nonzero coefficients of Q(T); the Hodge polygon of the basis has slope
 * n - m with multiplicity h_m (pole order m, Section 2.3), and lies below it
 * (Mazur).  Segments are reported left to right with integer rise over
 * length (the vertices are lattice points), collinear pieces merged.
 *   p_rank        length of the Newton segment whose slope is the least Hodge
 *                 slope (slope 0 for curves: the p-rank of the Jacobian;
 *                 slope 1 for cubic threefolds)
 *   ordinary      Newton polygon = Hodge polygon
 *   supersingular one slope, w/2 (w = n - 1 the weight)
 *   height        for Hodge numbers 1, b - 2, 1 around the middle slope w/2
 *                 (quartic K3 surfaces: the Artin-Mazur height; cubic
 *                 fourfolds: the Newton height): the h with first Newton slope
 *                 w/2 - 1/h; 0 = infinite (supersingular); -1 = not defined
 *   domino        surfaces (nvars = 4): the least vertical distance between
 *                 the Newton and the Hodge polygon over the slope-1 part of
 *                 the Hodge polygon, as domino_num / domino_den (0 = Hodge-
 *                 Witt); domino_num = -1 for other dimensions
 * lpoly: Q(T) as cr_frobenius_batch writes it ((b + 1) x 4 words, a_0 = 1),
 * b = the basis size of (nvars, degree).  CR_EINVAL for bad arguments or a
 * polynomial without a_0 = 1 or a nonzero a_b.
 */
#define CR_NEWTON_MAX 256
typedef struct {
    int32_t b;
    int32_t nseg;
    int32_t seg_len[CR_NEWTON_MAX];
    int32_t seg_rise[CR_NEWTON_MAX];
    int32_t p_rank;
    int32_t ordinary, supersingular;
    int32_t height;
    int32_t domino_num, domino_den;
} cr_newton;
cr_status cr_newton_polygon(int32_t nvars, int32_t degree, int32_t p, const int64_t *lpoly, cr_newton *out);

/* Device memory hook: where the batch workspaces and the cr_mlp handles get
 * their device memory (for instance a framework's caching allocator); without
 * one, hipMalloc / hipFree.  alloc(bytes, ctx) returns `bytes` of device
 * memory on the current device, 256-byte aligned, or NULL (the call then
 * fails with CR_ENOMEM); free_(ptr, ctx) takes back a block alloc returned.
 * Both NULL restores hipMalloc; exactly one NULL is CR_EINVAL.  The setting
 * is process-wide.  Installing it frees the library's cached workspaces (the
 * next call allocates through the new hook); every block is returned through
 * the hook that allocated it, and only after the device has finished all work
 * (the library waits for the device before calling free_), so a hook may hand
 * the block out again at once.  The hooks run on the thread that calls the
 * library, inside cr_frobenius_batch, cr_frobenius, cr_autotune, cr_release,
 * cr_set_allocator and the cr_mlp_* calls, and must not call back into the
 * library.  Pinned host staging still comes from hipHostMalloc, and
 * cr_frobenius_batch_noalloc allocates nothing through either. */
typedef void *(*cr_alloc_fn)(size_t bytes, void *ctx);
typedef void (*cr_free_fn)(void *ptr, void *ctx);
cr_status cr_set_allocator(cr_alloc_fn alloc, cr_free_fn free_, void *ctx);

/* Frees the library's cached device and host workspaces. */
cr_status cr_release(void);

/* Message of the last failure on the calling thread ("" if none). */
const char *cr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CRFROB_H */
