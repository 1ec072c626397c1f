/*
 * npcf.h -- C ABI of the MI355X (gfx950) separable N-point correlation
 * function estimator.
 *
 * The estimator is eq. NPCF-estimator-discrete of Philcox & Slepian,
 * "Efficient Computation of N-Point Correlation Functions in D Dimensions"
 * (arXiv:2106.10278), section "Application to Discrete Data":
 *
 *   zeta^{Lambda, b} = 1/V_D * sum_j w_j sum_{[l^1]..[l^{N-1}]} C^{Lambda;0} prod_i a^{b_i}_{[l^i]}(y_j)
 *   a^b_[l](y_j)     = 1/v_b * sum_k w_k Y*_[l](unit(y_k - y_j)) Theta^b(|y_k - y_j|)
 *
 * for isotropic (vec L = 0) basis states, N in {3, 4, 5}, D in {2, 3, 4}
 * (D = 4 with N = 3 only, N = 5 with D = 3 only), flat periodic or open boxes.  The harmonic stage
 * (the O(n^2) sum defining a) and the coupling stage (the per-primary sum
 * over [l] weighted by the coupling coefficients of eq. Coupling-C) run as
 * hand-written HIP kernels on the plan's stream.
 *
 * Conventions (fixed by the library, documented per call):
 *  - hyperspherical harmonics of Appendix A (eq. hypersph-def) with azimuth
 *    factor e^{+i l1 theta1}, theta1 = atan2(x2, x1), cos theta_K =
 *    x_{K+1}/|x_{1..K+1}|;
 *  - index sets |l1| <= l2 <= ... <= l_{D-1} <= lmax (eq. selection-rules);
 *  - coupling to vec L = 0 through the Clebsch-Gordan coefficients of eq.
 *    CG-examples (D = 2: Kronecker delta; D = 3: Wigner 3-j); for D = 4, N = 3
 *    the coupling of two states to zero is (-1)^{l3-l1}/sqrt((l3+1)^2); for
 *    N = 5 (section "Hydrodynamic Turbulence") the three-CG chain of eq.
 *    Coupling-C through the intermediate l12, i.e. that section's two-3j
 *    form with the prefactor sqrt(2 l12 + 1);
 *  - bins: e_b <= r < e_{b+1} on exact lattice distances; v_b the shell
 *    volume |S^{D-1}| (e_{b+1}^D - e_b^D)/D;
 *  - output: for D >= 3 the real part of zeta for even sum of the l_{D-1}
 *    and the imaginary part for odd (eq. basis-parity-conj: the other part
 *    vanishes for a real field); D = 2 outputs both parts.
 *
 * Positions are quantised on the device to the lattice box * q / 2^32
 * (q = round(x / box * 2^32) mod 2^32 per axis); inputs already on that
 * lattice are represented exactly.
 *
 * Thread safety: a plan is used by one host thread at a time; calls on one
 * plan are ordered on its stream.  No C++ exception crosses this ABI.
 */
#ifndef NPCF_H
#define NPCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NPCF_OK = 0,
    NPCF_E_INVALID = 1,      /* bad argument or configuration */
    NPCF_E_UNSUPPORTED = 2,  /* valid request outside what the library implements */
    NPCF_E_NOMEM = 3,        /* device or host allocation failed */
    NPCF_E_DEVICE = 4,       /* a HIP call failed (no GPU, launch failure, ...) */
    NPCF_E_STATE = 5         /* call out of order (e.g. after a failed accumulate) */
} npcf_status;

/* Coupling-stage arithmetic.  The harmonic stage always evaluates pair
 * geometry and harmonics in FP32 with exact integer periodic separations and
 * FP64 near-edge binning; long reductions are carried in FP64. */
typedef enum {
    NPCF_PLAIN_FP32 = 0,    /* coupling products in FP32 (MFMA f32) */
    NPCF_MIXED_BF16X3 = 1,  /* coupling GEMM in BF16 hi+lo split, 3 MFMA products, FP32 accumulate */
    NPCF_MIXED_FP16X3 = 2,  /* FP16 hi+lo split of power-of-two scaled operand tiles, 3 MFMA products */
    NPCF_MIXED_BF16X6 = 3   /* BF16 hi+mid+lo split, 6 MFMA products (FP32-level accuracy) */
} npcf_precision;

typedef enum {
    NPCF_NORM_RAW = 0,         /* eq. NPCF-estimator-discrete as written */
    NPCF_NORM_BY_RANDOMS = 1   /* divide each zeta^{Lambda,b} by the Lambda = 0 component of the
                                  randoms-only estimator (accumulated with NPCF_ROLE_RANDOMS) */
} npcf_norm;

typedef enum {
    NPCF_ROLE_DATA = 0,     /* accumulate into the estimator */
    NPCF_ROLE_RANDOMS = 1   /* accumulate into the randoms normalisation accumulator */
} npcf_role;

typedef enum {
    NPCF_BASIS_ISOTROPIC = 0,     /* vec L = 0: the isotropic basis (eq. Coupling-C) */
    NPCF_BASIS_LINE_OF_SIGHT = 1  /* D = 3, N = 3: P^{0L}_{l1 l2} (section "Large-Scale Structure"),
                                     line of sight along axis 3, labels (l1, l2, L), L <= Lmax */
} npcf_basis;

typedef enum {
    NPCF_GEOMETRY_FLAT = 0,      /* flat box (periodic or open) */
    NPCF_GEOMETRY_SPHERE = 1     /* points on the unit D-sphere, the constant-curvature space of section
                                    "Constant-Curvature Metric" with k = 1, chi(r) = sin r (eq. metric):
                                    D = 2 (the sky of section "Cosmic Microwave Background") or D = 3,
                                    N = 3 or 4, isotropic basis, lmax <= 5; positions are unit vectors
                                    in R^{D+1} (pos [D+1][n]); edges are geodesic angles in radians,
                                    0 < edges[0] with cos(edges[0]) < 1 - 1e-12 (so the self pair is
                                    in no bin), edges[nbins] <= pi; bins e_b <= theta < e_{b+1}
                                    decided on the FP64 dot product; the direction of a secondary is
                                    its tangent component at the primary p in the frame
                                    D = 2: e1 = unit(z x p) (unit(x x p) when |p_z| > 0.9), e2 = p x e1;
                                    D = 3: e1, e2, e3 = p i, p j, p k for p = a + b i + c j + d k, i.e.
                                    (-b, a, d, -c), (-c, -d, a, b), (-d, c, -b, a);
                                    v_b = |S^{D-1}| int_{e_b}^{e_{b+1}} sin^{D-1} r dr:
                                    D = 2: 2 pi (cos e_b - cos e_{b+1}), V = 4 pi;
                                    D = 3: 2 pi (d - cos(e_b + e_{b+1}) sin d), d = e_{b+1} - e_b,
                                    V = 2 pi^2; box and periodic are ignored; every secondary is
                                    visited (no cell list) */,
    NPCF_GEOMETRY_HYPERBOLIC = 2 /* points of hyperbolic space H^D, the constant-curvature space of section
                                    "Constant-Curvature Metric" with k = -1, chi(r) = sinh r (eq. metric),
                                    on the hyperboloid of R^{D,1}: D = 2 or 3, N = 3 or 4, isotropic
                                    basis, lmax <= 5; positions pos[D+1][n] with x0^2 - x1^2 - .. - xD^2
                                    = 1, x0 > 0; <x, y> = x0 y0 - x1 y1 - .. - xD yD; edges are geodesic
                                    distances, cosh(edges[0]) >= 1 + 1e-9, edges[nbins] <= 20; bins
                                    e_b <= theta < e_{b+1}, cosh theta = <p, q>, decided on the FP64
                                    product; the self pair is excluded by index; the direction of a
                                    secondary is its tangent component at p in the frame e_j(p) =
                                    (p_j, unit_j + p_j (p1..pD) / (1 + p0)) (the boost taking the origin to
                                    p applied to the axes), u_j = -<q, e_j(p)>; v_b = |S^{D-1}|
                                    int_{e_b}^{e_{b+1}} sinh^{D-1} r dr: D = 2: 2 pi (cosh e_{b+1} -
                                    cosh e_b); D = 3: 2 pi (cosh(e_b + e_{b+1}) sinh d - d), d =
                                    e_{b+1} - e_b; V = box[0], the volume of the region the catalogue
                                    fills (given by the caller); periodic is ignored; every secondary is
                                    visited (no cell list) */
} npcf_geometry;

typedef struct {
    int D;               /* dimension: 2, 3 or 4 */
    int N;               /* correlation order: 3, 4 or 5 (N = 4 needs D <= 3, N = 5 D = 3) */
    int lmax;            /* maximum l_{D-1}: D=2 <= 16, D=3 <= 10 (<= 5 for N = 5), D=4 <= 6 */
    int nbins;           /* radial bins, 1..16 */
    const double *edges; /* host, nbins+1 strictly increasing values, edges[0] > 0; copied */
    double box[4];       /* side length per axis (first D used), > 0; V_D = product */
    int periodic;        /* 1: periodic box, 0: open; either way 2 * edges[nbins] < every side
                            (separations are held as 32-bit lattice offsets) */
    int btuple_mode;     /* 0: b1 < b2 < ... (default); 1: every tuple (b1..b_{N-1} free) */
    int precision;       /* npcf_precision */
    int norm;            /* npcf_norm */
    int basis;           /* npcf_basis (0 for a zero-initialised config) */
    int Lmax;            /* NPCF_BASIS_LINE_OF_SIGHT: largest L, 0..2 lmax (ignored otherwise) */
    int geometry;        /* npcf_geometry (0, flat, for a zero-initialised config) */
} npcf_config;

typedef struct npcf_plan_s *npcf_plan_t;

/* Create a plan.  Validates cfg, enumerates the basis (Lambda labels and
 * radial tuples), builds the coupling tables (eq. Coupling-C) on the host in
 * FP64 and uploads them, and allocates device workspace for catalogues of up
 * to max_points points.  `stream` is a hipStream_t (NULL: the default
 * stream).  The plan owns all device memory it allocates.
 * Errors: NPCF_E_INVALID (bad cfg, max_points < 1, out == NULL, or no
 * radial tuple: btuple_mode 0 with fewer than N - 1 bins),
 * NPCF_E_UNSUPPORTED (N, D, lmax or nbins outside the table above),
 * NPCF_E_NOMEM, NPCF_E_DEVICE. */
npcf_status npcf_plan(const npcf_config *cfg, void *stream, int64_t max_points, npcf_plan_t *out);

/* Add the contribution of primaries [prim_begin, prim_end) (indices into the
 * catalogue) against all n secondaries of the same catalogue to the plan's
 * FP64 accumulator selected by `role` (eq. NPCF-estimator-discrete is a sum
 * over primaries, so calls over disjoint ranges add up).
 *  pos: device pointer, SoA double [D][n] (pos[k*n + i] = coordinate k of point i)
 *  w:   device pointer, double [n] (real weights)
 * The caller keeps pos and w valid until the plan's stream has passed this
 * call.  Asynchronous.  Errors: NPCF_E_INVALID (n < 1, n > max_points, empty or
 * out-of-range primary range, NULL pointers, bad role), NPCF_E_DEVICE.
 * Non-finite coordinates or weights set a device flag reported by the next
 * npcf_finalize as NPCF_E_INVALID. */
npcf_status npcf_accumulate(npcf_plan_t plan, const double *pos, const double *w, int64_t n,
                            int64_t prim_begin, int64_t prim_end, int role);

/* Gridded data (section "Application to Gridded Data"): the field X sampled
 * on a periodic grid of dims[0] x ... x dims[D-1] nodes covering the box
 * (node (i_0, ..) at x_k = i_k box_k / dims_k) is the catalogue of its nodes
 * with weights w = X dV (dV = prod box_k / dims_k), and a^b_[l] of every node
 * is computed for all nodes at once as the correlation of w with
 * conj(Y_[l]) Theta^b / v_b, by FFTs on the device (complex FP64, one pass per
 * axis).  The nodes [prim_begin, prim_end) (row-major node index, last axis
 * fastest) are then the primaries of the coupling stage, as in
 * npcf_accumulate; the result equals npcf_accumulate on the node catalogue up
 * to rounding.  The plan keeps the FFTs of the kernels for the last grid shape
 * (nbins x states x prod dims complex doubles, twice that while accumulating);
 * a new shape rebuilds them.
 *  field: device pointer, double [prod dims], row-major
 *  dims:  host pointer, int [D], each a power of two in 2..2048
 * The primary count per call is limited only by memory (chunks of up to
 * max_points rows).  Asynchronous after the first call on a shape.
 * Errors: NPCF_E_INVALID (NULL pointers, dims not powers of two, empty or
 * out-of-range node range, open box, bad role), NPCF_E_UNSUPPORTED (D = 4),
 * NPCF_E_NOMEM, NPCF_E_DEVICE.  Non-finite field values are reported by the
 * next npcf_finalize as NPCF_E_INVALID. */
npcf_status npcf_accumulate_grid(npcf_plan_t plan, const double *field, const int *dims, int64_t prim_begin,
                                 int64_t prim_end, int role);

/* Harmonic stage of the gridded path alone: a^b_[l] (eq. alm-bin-def,
 * including 1/v_b) of the nodes [prim_begin, prim_end), from the same FFTs as
 * npcf_accumulate_grid, written to `out` (host, double, (prim_end -
 * prim_begin) * nbins * n_state * 2 entries, layout as npcf_alm).  The node
 * pairs are counted as data pairs.  Synchronises.  Errors as
 * npcf_accumulate_grid, plus NPCF_E_INVALID when out_len is wrong. */
npcf_status npcf_alm_grid(npcf_plan_t plan, const double *field, const int *dims, int64_t prim_begin,
                          int64_t prim_end, double *out, size_t out_len);

/* Synchronise the plan's stream and write the finalised estimator to `out`
 * (host, double, out_len entries): zeta / (V_D prod_i v_{b_i}), parity part
 * as described above, optionally divided by the randoms normalisation.
 * Layout: out[lambda * n_bt + t] (D >= 3) or out[(lambda * n_bt + t) * 2 + {0: Re, 1: Im}]
 * (D = 2), Lambda and radial tuples in the order of npcf_describe.
 * Does not reset the accumulators.  Errors: NPCF_E_INVALID (out_len wrong,
 * out NULL, non-finite input seen, BY_RANDOMS with a zero randoms
 * normalisation), NPCF_E_DEVICE. */
npcf_status npcf_finalize(npcf_plan_t plan, double *out, size_t out_len);

/* Describe the output layout.  Any pointer may be NULL.
 *  n_lambda: number of Lambda labels; lambda_labels: int [n_lambda][3], [n_lambda][5] for N = 5
 *    (N=3, D>=3: (l,0,0); N=3, D=2: (l,-l,0); N=4: (l1,l2,l3), l12 = l3 implied for D = 3,
 *    l3 = -l1-l2 for D = 2; line-of-sight basis: (l1,l2,L), |l1-l2| <= L <= min(l1+l2, Lmax),
 *    Re part reported for even l1+l2+L, Im for odd; N = 5: (l1,l2,l12,l3,l4) with
 *    |l1-l2| <= l12 <= l1+l2 (not capped at lmax), |l12-l3| <= l4 <= min(l12+l3, lmax), Re
 *    reported for even l1+l2+l3+l4, Im for odd), lexicographic;
 *  n_bt: number of radial tuples; btuples: int [n_bt][3] (unused entries 0), [n_bt][4] for
 *    N = 5, lexicographic;
 *  out_len: entries npcf_finalize writes. */
npcf_status npcf_describe(npcf_plan_t plan, int *n_lambda, int *lambda_labels, int *n_bt, int *btuples,
                          size_t *out_len);

/* Number of ordered in-range pairs (e_0 <= r < e_nbins, i != j) seen by the
 * harmonic stage since the last reset, for each role (synchronises). */
npcf_status npcf_pair_count(npcf_plan_t plan, int64_t *pairs_data, int64_t *pairs_randoms);

/* Harmonic stage only (eq. alm-bin-def, discrete form): a^b_[l](y_j) for
 * primaries j in [prim_begin, prim_end), written to `out` (host, double,
 * (prim_end-prim_begin) * nbins * n_state * 2 entries,
 * out[((p * nbins + b) * n_state + s) * 2 + {Re, Im}]), including 1/v_b.
 * States are the stored half l1 >= 0 in the order: D=2: l = 0..lmax;
 * D=3: (l, m) l-major, m = 0..l; D=4: (l3, l2, l1) l3-major, l1 = 0..l2.
 * The others follow from a_{(-l1)..} = (-1)^{l1} conj(a_{l1..}) (D >= 3) or
 * a_{-l} = conj(a_l) (D = 2).  Synchronises.  Errors as npcf_accumulate,
 * plus NPCF_E_INVALID when out_len is wrong. */
npcf_status npcf_alm(npcf_plan_t plan, const double *pos, const double *w, int64_t n,
                     int64_t prim_begin, int64_t prim_end, double *out, size_t out_len);

/* Batched accumulation of `ncat` independent catalogues (the estimator of
 * eq. NPCF-estimator-discrete for each, every point a primary; e.g. many
 * data-plus-randoms catalogues of uneven sizes).
 * Catalogue c: pos[c] (device, SoA double [D][n[c]]) and w[c] (device,
 * double [n[c]]); data and randoms of one catalogue are one point set told
 * apart only by their weights.  All catalogues share one cell list (keys
 * catalogue-major) and run as one launch sequence: a persistent harmonic
 * kernel over rows of every catalogue, coupling blocks cut at catalogue
 * boundaries, one FP64 accumulator per catalogue.  Catalogues are taken
 * smallest first (ascending n[c], ties in index order), so that most of them
 * complete early (see npcf_finalize_batch's done_ms).  The sequence is captured
 * as a HIP graph the first time a shape (ncat, n[], pos[], w[]) is seen and
 * replayed afterwards; device workspace for the batch is allocated then
 * (independent of max_points).  Asynchronous: ordered after the plan's stream
 * and the plan's stream waits for it.  The caller's buffers must stay valid
 * and unchanged in address while the shape is reused.  Not available with
 * NPCF_NORM_BY_RANDOMS (NPCF_E_UNSUPPORTED).
 * Errors: NPCF_E_INVALID (null pointers, ncat < 1, n[c] < 1, more than 2^31
 * points in total), NPCF_E_UNSUPPORTED (too many cells for 32-bit keys),
 * NPCF_E_NOMEM, NPCF_E_DEVICE, NPCF_E_STATE. */
npcf_status npcf_accumulate_batch(npcf_plan_t plan, int ncat, const double *const *pos, const double *const *w,
                                  const int64_t *n);

/* Finalised output of catalogue `cat` of the last npcf_accumulate_batch,
 * with the layout and rules of npcf_finalize (synchronises).  *done_ms (may
 * be NULL): that catalogue's completion time in milliseconds after the start
 * of the batch, from device-clock timestamps written in the launch sequence;
 * *pairs (may be NULL): its in-range ordered pair count.
 * Errors: NPCF_E_INVALID (cat out of range, out_len wrong, non-finite input),
 * NPCF_E_STATE (no batch run yet). */
npcf_status npcf_finalize_batch(npcf_plan_t plan, int cat, double *out, size_t out_len, double *done_ms,
                                int64_t *pairs);

/* npcf_accumulate for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, hosts that forbid allocation):
 * the same computation, arguments, accumulators and errors as
 * npcf_accumulate, but every per-call device buffer (quantised positions,
 * cell list, rows of a, coupling partials, work counter) is cut from one
 * static device workspace of 64 MiB that the library holds on each device it
 * runs on until the process ends; the call makes no device or host memory
 * allocation and records no timing events (npcf_stage_ms does not see it).
 * The workspace used is that of the device that was current when the plan
 * was made (npcf_plan looks up its address).  Primaries are processed in chunks that fit the
 * workspace, so results agree with npcf_accumulate up to rounding order.
 * Every call on a device shares that device's workspace and leaves its
 * contents behind (each call rewrites what it reads): calls that overlap in
 * time on one device, from any plans or streams, race and give wrong results.
 * Flat geometry only.  Errors: as npcf_accumulate; NPCF_E_INVALID also when
 * the catalogue does not fit the workspace (about 17 MB per 256k points in
 * D = 3 besides the cell grid and one 16-row chunk; the detail names the bytes
 * needed), NPCF_E_UNSUPPORTED for the sphere geometry, NPCF_E_DEVICE when the
 * workspace could not be found on the device. */
npcf_status npcf_accumulate_static(npcf_plan_t plan, const double *pos, const double *w, int64_t n,
                                   int64_t prim_begin, int64_t prim_end, int role);

/* Zero the accumulators and pair counters (asynchronous). */
npcf_status npcf_reset(npcf_plan_t plan);

/* Release the plan and its device memory (synchronises first). NULL is a no-op. */
npcf_status npcf_destroy(npcf_plan_t plan);

/* Tuning knobs (0 keeps the current value): cell subdivision s (flat cells
 * of side >= r_max / s, eight times thinner along x, the axis of a stencil
 * row; 1..8), primaries per coupling block (rounded up to a
 * multiple of 16), and primaries per chunk (rows of a^b held at once; at most
 * the size chosen at plan time).  Synchronises; takes effect on the next
 * accumulate (a batch shape is captured again).  Errors: NPCF_E_INVALID
 * (out of range), NPCF_E_NOMEM. */
npcf_status npcf_set_tuning(npcf_plan_t plan, int cell_subdiv, int couple_block, int64_t chunk_rows);

/* Tile shapes and launch sizes of a plan (npcf_get_tuning, npcf_apply_tuning). */
typedef struct {
    int cell_subdiv;             /* cells of side >= r_max / s (x eight times thinner), 1..8 */
    int couple_block;            /* primaries per coupling block (multiple of 16; 0: the automatic rule) */
    int64_t chunk_rows;          /* primaries per chunk (rows of a held at once) */
    int harmonic_blocks_per_cu;  /* persistent harmonic grid: blocks of four waves per compute unit, 1..32 */
    int curved_bins_per_pass;    /* curved geometries: radial bins per pass of the all-pairs kernel, one of the
                                    two widths compiled for the plan's D and lmax, the narrower by default
                                    (npcf_get_tuning reports the current one; 0 on the flat geometry, and 0
                                    keeps it) */
} npcf_tuning;

/* The plan's current tuning (the automatic values where nothing was set).
 * Errors: NPCF_E_INVALID (NULL arguments). */
npcf_status npcf_get_tuning(npcf_plan_t plan, npcf_tuning *out);

/* Set every knob of `t` that is non-zero (as npcf_set_tuning, plus the
 * harmonic grid and the curved-space bins per pass).  Synchronises.  Errors:
 * NPCF_E_INVALID (out of range; bins per pass on a flat plan or not one of
 * the plan's two widths), NPCF_E_NOMEM. */
npcf_status npcf_apply_tuning(npcf_plan_t plan, const npcf_tuning *t);

/* Autotuner for the given catalogue (positions and weights as npcf_accumulate):
 *  - flat geometry: the cell subdivision s = 1..6 (1..4 for D = 4) and then the harmonic
 *    grid's blocks per CU (2, 3, 4, 6, 8), timing the harmonic stage with its
 *    cell list on four ranges spread over the catalogue of
 *    max(sample / 4, min(n / 16, 131072)) primaries each: enough rows to
 *    fill the persistent grid many times over, so that the timing follows
 *    throughput rather than the latency of single rows;
 *  - curved geometries (no cell grid): the bins per pass of the all-pairs
 *    kernel, its two widths timed on the whole catalogue;
 *  - the primaries per coupling block (the automatic rule, 256, 512, 1024,
 *    2048) and the chunk rows (the plan's largest, or n / 32), timing the
 *    coupling and the whole pass on the whole catalogue, whose launches are
 *    the ones tuned (on a part of it a block size gives another block count);
 *  each by the best of two runs (HIP events); a setting other than the
 *  default must win by 2%.  The choice is applied to the plan (read it with
 *  npcf_get_tuning).  With the environment variable NPCF_TUNE_CACHE naming a
 *  file, a tuning stored there for the same problem (D, N, lmax, bins, r_max,
 *  n, box, precision, b-tuple mode, basis, periodicity, geometry, CU count) is applied
 *  without timing, and a new one is written to it (JSON).  Resets the
 *  accumulators.  Outputs (may be NULL): the chosen subdivision, block size
 *  (0: the automatic rule) and the timed ms of harmonic + coupling.  Errors
 *  as npcf_accumulate. */
npcf_status npcf_autotune(npcf_plan_t plan, const double *pos, const double *w, int64_t n, int64_t sample,
                          int *cell_subdiv, int *couple_block, double *best_ms);

/* Device time in milliseconds, accumulated since the last reset and measured
 * with HIP events on the plan's stream, of ms3[0] the harmonic stage,
 * ms3[1] the coupling stage with its FP64 reduction and ms3[2] the cell-list
 * build (synchronises). */
npcf_status npcf_stage_ms(npcf_plan_t plan, double *ms3);

/* Static description of a status code (never NULL). */
const char *npcf_strerror(npcf_status status);

/* Detail of the last failure on the calling thread: for NPCF_E_DEVICE or
 * NPCF_E_NOMEM the HIP error name and code and the failing call; for an
 * NPCF_E_UNSUPPORTED from npcf_plan the setting it rejected, where one is
 * named ("" if none; never NULL; npcf_plan clears it on entry; valid until
 * the next failure on this thread). */
const char *npcf_last_error_detail(void);

/* Library version string (never NULL). */
const char *npcf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NPCF_H */
