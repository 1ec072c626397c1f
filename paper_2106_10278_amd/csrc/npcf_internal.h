// Internal declarations shared by the host planner and the HIP kernels of the
// NPCF library.  Nothing here is part of the public ABI (include/npcf.h).
#pragma once
#include <cstddef>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "npcf.h"

namespace npcf {

constexpr int kMaxD = 4;
constexpr int kMaxBins = 16;
constexpr int kWave = 64;

// Number of stored harmonic states (l1 >= 0 half) for dimension D and lmax L.
//   D = 2: l = 0..L                       -> L + 1
//   D = 3: (l, m), 0 <= m <= l <= L        -> (L+1)(L+2)/2
//   D = 4: (l3, l2, l1), 0 <= l1 <= l2 <= l3 <= L -> sum_{l3} (l3+1)(l3+2)/2
__host__ __device__ constexpr int stored_states(int D, int L)
{
    return D == 2 ? L + 1
         : D == 3 ? (L + 1) * (L + 2) / 2
                  : (L + 1) * (L + 2) * (L + 3) / 6;
}

// FP64 product and sum, each rounded on its own.  HIP's __dmul_rn and
// __dadd_rn are the plain operators, which the compiler fuses into an FMA
// under its default contraction; the pragma keeps these apart, so a squared
// distance or a dot product takes the definition's arithmetic (as the FP64
// oracle, built without FMA, does) and a bin is decided exactly as there.
__device__ __forceinline__ double mul_rn(double x, double y)
{
#pragma clang fp contract(off)
    return x * y;
}

__device__ __forceinline__ double add_rn(double x, double y)
{
#pragma clang fp contract(off)
    return x + y;
}

// ---------------------------------------------------------------------------
// Device workspace of one catalogue after the cell-list build.
// ---------------------------------------------------------------------------
struct CellList {
    uint32_t *q[kMaxD] = {nullptr, nullptr, nullptr, nullptr};  // sorted lattice coordinates (SoA)
    float *w = nullptr;               // sorted weights (FP32)
    double *w64 = nullptr;            // sorted weights (FP64)
    int32_t *orig = nullptr;          // sorted position -> original index
    uint32_t *cell_start = nullptr;   // [ncell + 1]
    int ncs[kMaxD] = {1, 1, 1, 1};    // cells per side
    int64_t ncell = 0;
};

// ---------------------------------------------------------------------------
// Harmonic stage arguments.
// ---------------------------------------------------------------------------
struct HarmArgs {
    const uint4 *rec;         // sorted packed records: D=2 (q0,q1,w,0), D=3 (q0,q1,q2,w), D=4 (q0..q3)
    const float *w;           // sorted weights (FP32)
    const uint32_t *cell_start;
    const int32_t *prim;      // sorted positions of this chunk's primaries
    int nrows;
    int nb;
    int ncs[kMaxD];
    double cell_len[kMaxD];   // cell side, lattice units (2^32 / ncs)
    double inv_cell_len[kMaxD];
    double rmax_lat[kMaxD];   // r_max in lattice units per axis
    double scale64[kMaxD];    // physical length of one lattice unit per axis
    float scale[kMaxD];
    float e2lo_f, e2hi_f;     // conservative FP32 range test on r^2 (physical)
    float bucket_lo, bucket_inv;  // r^2 -> bucket index for the first bin guess
    int nbucket;
    const double *e2;         // [nb + 1] squared edges (physical, FP64)
    const uint8_t *bucket_bin;  // [nbucket] bin at the low end of each r^2 bucket
    float *A;                 // out: [nrows][nb][2 * nstate]
    float *wrow;              // out: [nrows] primary weights
    unsigned long long *pairs;  // in-range pair counters, one per catalogue
    unsigned int *work;       // dynamic row counter (zeroed before launch)
    int periodic;
    // batches: several catalogues sorted catalogue-major into one cell list.
    // cat_begin[c] is catalogue c's first sorted position ([ncat + 1]); its
    // cells are cell_start[c * ncell_cat ...].  nullptr: a single catalogue.
    const int64_t *cat_begin;
    int ncat;
    int64_t ncell_cat;
    int per_bin;              // 1: one pass per radial bin (k_harmonic_pass) where the instance has it
    int cube;                 // 1: every axis has the same lattice scale (a periodic cube)
};

// ---------------------------------------------------------------------------
// Factorised N = 4, D = 3 coupling.  For a pair (l1, l2) and m3 >= 0 the
// products P_{m1} = op(a_{l1 |m1|}[b1]) op(a_{l2 |m2|}[b2]) (m2 = -m1 - m3) are
// shared by every l3 of the pair; S_{l3} = sum_{m1} coef(l3, m1) P_{m1} for each
// output slot (one slot per l3 of the pair, in increasing l3).
constexpr int kMaxSlots = 6;   // l3 values of one (l1, l2) pair at lmax <= 10 is at most 11; 6 covers lmax <= 5
struct FProd {
    int16_t s1, s2;      // stored state indices
    int8_t conj1, conj2;
    int16_t pad;
};
// coefficients per product in the factorised table: the slots of one product
// are adjacent and 32-byte aligned (one wide scalar load)
constexpr int kFCoefStride = 8;
static_assert(kFCoefStride >= kMaxSlots, "a product holds every slot coefficient");
// jobs (pair, tile) per wave of the factorised N = 4 coupling kernel
constexpr int kFJobsPerWave = 1;

struct FGroup {          // one (pair, m3)
    int prod_begin, prod_end;
    int coef_begin;      // coef[coef_begin + (t - prod_begin) * kFCoefStride + slot]
    int slot_mask;       // slots with l3 >= m3: slots [0, nact) (a pair's slots run by falling l3)
    int nact;            // number of active slots
    int16_t s3[kMaxSlots];  // state of leg 3 for each slot: (l3, m3)
};
// the coupling kernel reads FProd as one uint2 and FGroup::s3 as dwords
static_assert(sizeof(FProd) == 8, "FProd is read as one uint2");
static_assert(offsetof(FGroup, s3) % 4 == 0 && sizeof(FGroup) % 4 == 0, "FGroup::s3 is read as dwords");
struct FPair {
    int grp_begin, grp_end;
    int nslot;
    int lam[kMaxSlots];  // Lambda index of each slot
    int part[kMaxSlots]; // 0: Re, 1: Im
};

// ---------------------------------------------------------------------------
// Isotropic 5PCF (D = 3, N = 5).  With M = m1 + m2 (folded to M >= 0):
//   zeta = sgn * sum_i w_i sum_{M >= 0} Re( S~_M[i](b1, b2) T~_M[i](b3, b4) )
//   S~_M = (-i)^{rot} h_M sum_{m1} (l1 l2 l12; m1, M-m1, -M) a_{l1 m1}[b1] a_{l2, M-m1}[b2]
//   T~_M = (-i)^{rot} (-1)^{l3+l4} sum_{m3} (l12 l3 l4; M, m3, -M-m3) a_{l3 m3}[b3] a_{l4, -M-m3}[b4]
// A job is (l12, beta = b2, group of S labels, group of <= kC5Cols columns):
// GEMM rows (S label, b1), columns (T label, (b3, b4)), K = primaries x {re, im}
// per M, every computed entry an output of the b-tuple order.
// ---------------------------------------------------------------------------
constexpr int kC5Rows = 128;   // GEMM rows of one job (8 tiles)
constexpr int kC5Cols = 64;    // GEMM columns of one job (one 16-column tile per wave)
constexpr int kC5Stride = 36;  // floats per staged row/column of S~ / T~ (32 K values + pad)
constexpr int kLmax5 = 5;
struct C5Label {   // one S label (l1, l2 | l12) or T label (l3, l4 | l12)
    int mt;        // terms of M: c5terms[c5mterm[mt + M] .. c5mterm[mt + M + 1]), M = 0..l12
    int rot;       // 1: multiply by -i (odd l1 + l2, resp. l3 + l4)
};
// A term in 8 bytes: x = s1 | s2 << 8 | conj1 << 16 | conj2 << 17, y = coef (FP32 bits).
// The labels of one l12 are consecutive and each holds l12 + 2 entries of
// c5mterm, so a job's labels own one contiguous run of c5mterm and of c5terms.
struct C5Job {
    int l12, beta;
    int nb1;                 // b1 values of each S label (b1 < nb1)
    int s_begin, ns;         // S labels [s_begin, s_begin + ns)
    int t_begin;             // first T label of this l12
    int col_begin, ncol;     // columns [col_begin, col_begin + ncol): T label col / npair, pair col % npair
    int pair_begin, npair;   // (b3, b4) pairs of this beta: c5pairs[pair_begin ..)
    int nrt;                 // row tiles: ceil(ns * nb1 / 16) <= 8
    int tile_begin;          // output tiles tile_begin + rt * 4 + ct
};

// ---------------------------------------------------------------------------
// Coupling stage arguments.
// ---------------------------------------------------------------------------
// One coupling term of a (Lambda, group) GEMM K-slice: S += coef * op1(a[s1]) * op2(a[s2]).
struct CoupleTerm {
    int16_t s1, s2;     // stored state indices
    int8_t conj1, conj2;
    int16_t pad;
    float coef;
};

// A group is one (Lambda, m3) pair for N = 4 (the contraction partner a3 =
// a[s3], conjugated when conj3) and one Lambda for N = 3.
struct CoupleGroup {
    int term_begin, term_end;   // N = 4: into the term table
    int s3;                     // N = 4: state of leg 3; N = 3: first state of l
    int nst;                    // N = 3: number of stored states of l
    int conj3;
    float scale3;               // N = 3: coefficient (f * sign / sqrt(dim)); N = 4: unused
};

struct CoupleArgs {
    const float *A;            // [nrows][nb][2 * nstate]
    const float *wrow;         // [nrows]
    int nrows;
    int nb;
    int nstate;
    int rows_per_block;        // primaries per workgroup (multiple of 16)
    int n_rowblocks;
    int nlam;
    int lam_per_block;
    const CoupleTerm *terms;
    const CoupleGroup *groups;
    const int *lam_group_begin;   // [nlam + 1] groups of each Lambda
    const int *lam_part;          // [nlam] 0: Re, 1: Im, 2: both (D = 2)
    const int2 *row_pairs;        // [mrows] (b1, b2) of GEMM row m (N = 4); unused for N = 3
    int mrows;                    // valid GEMM rows (N = 4)
    int mtiles;                   // ceil(mrows / 16) (N = 4); 1 (N = 3)
    int max_block_terms;          // N = 4: most terms any block's jobs use (LDS copy)
    double *partial;              // out: [n_rowblocks][njobs][16][16]
    // batches: rows [rb_begin[rb], rb_end[rb]) of row block rb (blocks never
    // straddle two catalogues); nullptr: blocks of rows_per_block rows
    const int *rb_begin;
    const int *rb_end;
    // factorised N = 4, D = 3 (nullptr: term-by-term kernel)
    const FPair *fpairs;
    const FGroup *fgroups;
    const FProd *fprods;
    const float *fcoef;
    const int2 *ftasks;          // per wave: two jobs (pair * mtiles + tile), -1 for none
    int nftasks;
    // N = 3 with a term list per Lambda (line-of-sight basis): one group per
    // Lambda, terms (s1, conj1, s2, conj2, coef) pairing a[b1] with a[b2]
    int n3_terms;
    // N = 5 (see C5Job); the output tiles are the "jobs" of the partial layout
    const C5Job *c5jobs;
    int nc5jobs;
    const C5Label *c5labels;
    const int *c5mterm;
    const uint2 *c5terms;
    const int2 *c5pairs;
    int c5_lds_extra;            // bytes of the largest job's term tables in LDS
};

// ---------------------------------------------------------------------------
// Gridded-data estimator (npcf_grid.hip).
// ---------------------------------------------------------------------------
struct GridArgs {
    int dims[3];
    int64_t ng;
    double h[3];            // grid spacing per axis
    const double *e2;       // [nb + 1] squared edges (device)
    int nb;
};

// ---------------------------------------------------------------------------
// Points on the unit 2-sphere (npcf_sphere.hip).
// ---------------------------------------------------------------------------
constexpr int kLmaxSphere = 5;   // larger l would spill the per-lane bin sums
// curved spaces: sorted secondaries per chunk (one per lane) of the all-pairs
// kernel's scan, each with a bounding cap
constexpr int kSphChunk = 64;

// real slots per bin of the all-pairs kernel: 2 per stored state (the
// imaginary slots of real states stay 0)
constexpr int sph_slots(int D, int L) { return D == 2 ? 2 * (L + 1) : (L + 1) * (L + 2); }

// bins per pass of the all-pairs kernel: as many as keep the lanes' FP32 sums
// (one per slot and bin) within a register budget, at least 1, at most 16 and
// at most 128 values in all (two per lane after the fold).  Two budgets, one
// kernel each, chosen per plan: wide (50 values on D = 2, 128 on D = 3; fewer
// passes, so fewer scans of the points) and narrow (10 and 42, one bin per
// pass from lmax 2 on D = 2 and lmax 5 on D = 3; fewer masked
// sums per pair, more waves per SIMD, and at one bin per pass no bucket
// table).  Which wins depends on the catalogue and the bins; the autotuner
// times both (in the current kernel the narrow one wins on the uniform
// 2-sphere, 25.6 against 27.2 ms, the clustered 3-sphere and H^3).
constexpr int sph_group(int D, int L, bool narrow)
{
    const int budget = narrow ? (D == 2 ? 10 : 42) : (D == 2 ? 50 : 128);
    const int g = budget / sph_slots(D, L);
    const int g1 = g < 1 ? 1 : (g > 16 ? 16 : g);
    return g1 * sph_slots(D, L) <= 128 ? g1 : 128 / sph_slots(D, L);
}

struct SphereArgs {
    const double *pos;          // [D + 1][n] unit vectors (sphere) or hyperboloid points (H^D)
    const double *w;            // [n]
    float4 *pf;                 // scratch [n]: S^2 (x, y, z, w), S^3 the coordinates, in FP32, written by launch_sphere
    int64_t n;
    int64_t p0;                 // primary of row 0: rows [0, rows) are primaries p0 + [0, rows)
    int rows;
    int nb;
    int group;                  // bins per pass: sph_group(D, L, false) or sph_group(D, L, true)
    double cedge[kMaxBins + 1]; // the edges' cosines: cos e (sphere) or -cosh e (H^D), decreasing
    unsigned *x0max;            // scratch word: largest x0 of the catalogue (H^D), written by launch_sphere
    // secondaries in spatial order (Hilbert cells), written by launch_sphere:
    // FP64 coordinates [D + 1][n], FP64 weights, original index, and per tile
    // of kSphChunk points a bounding cap (centre [4], radius in geodesic distance)
    double *spos;
    double *sw;
    int32_t *sorig;
    float *caps;                // [ntiles][8]
    uint32_t *key, *count, *cell_start, *cursor, *scan;  // sort scratch (cells: ncell + 1)
    int32_t *perm;
    int64_t scan_len;
    int ncell_bits;             // bits per axis of the Hilbert cells
    unsigned *bbox;             // [8] ordered-float min/max of the key axes (H^D)
    // the primaries p0 + [0, rows) in the same spatial order (positions in it),
    // so that the waves of a block take nearby primaries and meet similar
    // tiles: prim [rows], and the compaction's flags and offsets [n]
    int32_t *prim;
    uint32_t *pflag, *ppos;
    float erad[kMaxBins + 1];   // the edges (geodesic distance), for the tile test
    float *A;                   // out: [rows][nb][2 nstate]
    float *wrow;                // out: [rows]
    unsigned long long *pairs;  // in-range pair counter
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t launch_quantize(int D, int periodic, const double *pos, const double *w, int64_t n, const double *box,
                           const int *ncs, uint32_t *const qtmp[kMaxD], uint32_t *cell, uint32_t *count, int *bad,
                           hipStream_t s);
// batches: quantise every catalogue's points into one array (global index g =
// off[c] + i) with cell key c * ncell_cat + cell, and copy the FP64 weights
hipError_t launch_quantize_batch(int D, int periodic, int ncat, const double *const *pos, const double *const *w,
                                 const int64_t *off, int64_t ntot, const double *box, const int *ncs,
                                 int64_t ncell_cat, uint32_t *const qtmp[kMaxD], double *wall, uint32_t *cell,
                                 uint32_t *count, int *bad, hipStream_t s);
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s);
// device clock (constant-rate wall clock) at this point of the stream into *ts
hipError_t launch_timestamp(unsigned long long *ts, hipStream_t s);
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *scratch,
                                 int64_t scratch_len, hipStream_t s);
hipError_t launch_scatter_perm(int64_t n, const uint32_t *cell, uint32_t *cursor, int32_t *perm, hipStream_t s);
hipError_t launch_cellsort(int64_t n, const uint32_t *cell, const uint32_t *cell_start, const int32_t *perm,
                           int32_t *perm_sorted, hipStream_t s);
hipError_t launch_gather(int D, int64_t n, const int32_t *perm_sorted, uint32_t *const qtmp[kMaxD],
                         const double *w, uint4 *rec, float *ws, double *w64s, int32_t *orig, hipStream_t s);
hipError_t launch_primlist(int64_t n, const int32_t *orig, int64_t p0, int64_t p1, uint32_t *flag,
                           uint32_t *pos_out, int32_t *prim, uint32_t *scratch, int64_t scratch_len, hipStream_t s);
hipError_t launch_harmonic_d2(int L, const HarmArgs &a, int grid, hipStream_t s);
hipError_t launch_harmonic_d3(int L, const HarmArgs &a, int grid, hipStream_t s);
hipError_t launch_harmonic_d4(int L, const HarmArgs &a, int grid, hipStream_t s);
int harmonic_lds_bytes_d2(int L);
int harmonic_lds_bytes_d3(int L);
int harmonic_lds_bytes_d4(int L);
int couple_njobs(int N, int nlam, int nparts, int mtiles);
int couple_jobs_per_block();
int couple_ftask_groups(int nftasks);
int couple_nblocks(int njobs, int nrb);
hipError_t launch_couple_kernel(int N, int precision, const CoupleArgs &a, int njobs, int nparts, const float *sfac,
                                hipStream_t s);
hipError_t launch_reduce_partials(const double *partial, int nrb, int64_t len, double *acc, hipStream_t s);
hipError_t launch_finalize2(const double *acc, const double *acc_rand, int nlam, int nparts, int mtiles,
                            const int *bt_row, const int *bt_col, const double *bt_scale, int nbt, int norm_by_randoms,
                            int lam0, double *out, int *bad, hipStream_t s);
// gridded data: kernel grids K'_{b,s} (zero-filled first), one FFT axis pass,
// node weights, node rows of a, a device counter increment
hipError_t launch_grid_kernel(int D, int L, const GridArgs &g, double2 *kern, int64_t nkern, hipStream_t s);
int fft_lines_per_block(int n);
int fft_lds_bytes(int n);
hipError_t launch_fft(const double2 *src, double2 *dst, const double2 *tw, int n, int64_t stride, int64_t total,
                      int inverse, const double2 *premul, int64_t ng, hipStream_t s);
hipError_t launch_grid_weights(const double *field, int64_t ng, double dV, double *w64, float *w32, double2 *xin,
                               int *bad, hipStream_t s);
hipError_t launch_grid_rows(const double2 *a, int64_t ng, int nbs, int nst, const uint8_t *sreal, const float *w32,
                            int64_t r0, int rows, float *A, float *wrow, hipStream_t s);
hipError_t launch_add_u64(unsigned long long *p, unsigned long long v, hipStream_t s);
hipError_t launch_sphere(int D, int L, int K, const SphereArgs &a, hipStream_t s);
// finalize from an accumulator index per output (N = 5): out[lam * nbt + t] =
// acc[idx[lam * nbt + t]] * sign[lam] * bt_scale[t] (optionally over the randoms' Lambda = 0)
hipError_t launch_finalize_idx(const double *acc, const double *acc_rand, const int *idx, const double *sign,
                               const double *bt_scale, int nlam, int nbt, int norm_by_randoms, int lam0, double *out,
                               int *bad, hipStream_t s);
int couple5_lds_bytes(int nb, int nstate, int extra);
hipError_t launch_couple5(int precision, const CoupleArgs &a, int ntiles, hipStream_t s);

// ---------------------------------------------------------------------------
// Host planner (npcf_plan.cpp)
// ---------------------------------------------------------------------------
struct Tables {
    int nstate = 0;
    std::vector<int> state_lab;        // [nstate][3]: (l1, l2, l3) as applicable
    std::vector<int> lam_lab;          // [nlam][lab_w]
    std::vector<int> bt_lab;           // [nbt][bt_w]
    int lab_w = 3, bt_w = 3;           // 5 and 4 for N = 5
    int nlam = 0, nbt = 0, nparts = 1;
    std::vector<int> lam_part;         // [nlam]
    std::vector<CoupleTerm> terms;
    std::vector<CoupleGroup> groups;
    std::vector<int> lam_group_begin;  // [nlam + 1]
    std::vector<int2> row_pairs;       // N = 4 GEMM rows
    int mrows = 0, mtiles = 1;
    std::vector<int> bt_row, bt_col;
    std::vector<double> bt_scale;
    std::vector<float> sfac;           // [nstate] N = 3 state factors
    std::vector<double> e2;            // [nb + 1]
    std::vector<uint8_t> bucket_bin;
    float bucket_lo = 0.f, bucket_inv = 0.f;
    float e2lo_f = 0.f, e2hi_f = 0.f;
    std::vector<double> vb;            // bin volumes (sphere: annulus areas)
    bool sphere = false;               // a curved space, every secondary visited (no cell list)
    int curv = 0;                      // its curvature sign: +1 the unit D-sphere, -1 hyperbolic space H^D
    std::vector<double> cedge;         // curved: the edges' cosines, cos e or -cosh e (decreasing)
    int lam0 = 0;
    // factorised N = 4, D = 3 coupling (empty otherwise)
    std::vector<FPair> fpairs;
    std::vector<FGroup> fgroups;
    std::vector<FProd> fprods;
    std::vector<float> fcoef;
    std::vector<int2> ftasks;
    bool n3_terms = false;             // N = 3 coupling from a term list (line-of-sight basis)
    // N = 5 (empty otherwise)
    std::vector<C5Label> c5labels;
    std::vector<int> c5mterm;
    std::vector<CoupleTerm> c5terms;
    std::vector<uint2> c5packed;       // c5terms in the 8-byte device form
    int c5_lds_extra = 0;
    std::vector<int2> c5pairs;
    std::vector<C5Job> c5jobs;
    int c5tiles = 0;                   // output tiles (accumulator = c5tiles x 256 doubles)
    std::vector<int> c5idx;            // [nlam][nbt] accumulator index of each output
    std::vector<double> c5sign;        // [nlam]
};

// Validates cfg and fills the tables; returns NPCF_OK or an error code and a message.
npcf_status build_tables(const npcf_config &cfg, Tables &t, std::string &err);
double clebsch_gordan(int j1, int m1, int j2, int m2, int J, int M);
double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);
// stored state index: D = 2: l; D = 3: (l = l2, m = l1); D = 4: (l3, l2, l1)
int state_index(int D, int l1, int l2, int l3);
// factorised D = 3, N = 4 coupling tables (npcf_plan4.cpp); left empty when a pair's l3 values exceed the slots
void build_factorised(Tables &t, int L);
// N = 5 tables (npcf_plan5.cpp); false when the outputs exceed the index range
bool build_c5(Tables &t, int L, int nb, int mode);

}  // namespace npcf
