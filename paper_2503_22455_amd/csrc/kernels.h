// Host-side launch wrappers of the HIP kernels (one declaration per kernel family).
#pragma once

#include "common.h"

namespace iim {

// ---- setup (setup.hip) -----------------------------------------------------
// Classify every node of the full grid of levels 0..nl-1 (two launches, no
// atomics): bbox[8 l ..] = {min x,y,z, max x,y,z} of level l's unknowns and,
// at [8 l + 6], != 0 when the body touches the box; count[l] = its unknowns.
// d_part: classify_part_ints(nl) ints of scratch.
constexpr int MAX_LEVELS = 16;  // multigrid levels of a problem
constexpr int CLASSIFY_BLOCKS = 512;
struct GeomSet {
    Geom g[MAX_LEVELS];
};
int classify_part_ints(int nl);
void run_classify_levels(const GeomSet& G, int nl, int* d_part, int* d_bbox, unsigned long long* d_count,
                         hipStream_t s);
// the levels of a problem, for kernels that treat all of them in one launch
// (blockIdx.y = level); off[l] = offset of level l in a per-level flag array
struct LevelSet {
    Geom g[MAX_LEVELS];
    Box b[MAX_LEVELS];
    uint8_t* labels[MAX_LEVELS];
    int64_t off[MAX_LEVELS];
};
// labels of every level's storage box
void run_box_labels(const LevelSet& S, int nl, hipStream_t s);
// crossing flags of every axis: flags[a * N + l] = 1 if the segment (l, l + e_a)
// carries a control point (N = box size)
void run_cp_flags(const Geom& g, const Box& b, const uint8_t* labels, uint8_t* flags, hipStream_t s);
// Flagged selections: out = indices (0..n-1) of the nonzero flags in increasing
// order, *count = their number; up to SEL_MAX selections in three launches,
// stream ordered, no host wait; d_part: SEL_BLOCKS * k ints of scratch.
constexpr int SEL_MAX = 20, SEL_BLOCKS = 1024;
struct SelItem {
    const uint8_t* flags;
    int64_t n;
    int32_t* out;
    int64_t* count;
};
struct SelSet {
    SelItem it[SEL_MAX];
};
void select_flagged_multi(const SelItem* items, int k, int* d_part, hipStream_t s);

struct CPDev {
    int64_t ncp;
    int nsides;
    int axis_start[4];   // cps of axis d: [axis_start[d], axis_start[d+1])
    int32_t* lower;      // local index of the lower node of the segment
    int32_t* axis;
    int32_t* a;          // [nsides][ncp] local index of the side's adjacent unknown
    int32_t* dir;        // [nsides][ncp] step from that node towards Gamma
    double* x;           // [3][ncp]
    double* n;           // [3][ncp]
    double* kappa;       // [ncp]
};
void run_cp_compute(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp,
                    int* d_err, hipStream_t s);

// high-order irregular nodes (level 0)
// (w = stencil half-width: nodes whose stencil reaches another side or the box)
void run_ho_irr_flag(const Geom& g, const Box& b, uint8_t* labels, uint8_t* flags, int w, hipStream_t s);
void run_ho_irr_records(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp,
                        const int32_t* nodes, int64_t nirr, int32_t* slots, int32_t* irr_index, int w,
                        int* d_err, hipStream_t s);

// Shortley-Weller rows: flags of the irregular unknowns of every level (at
// flags + S.off[l]), then per level their rows
// rec[k * (1 + 2 dim)] = {diag, coefficient of neighbour (d, -), (d, +), ...} scaled by h^2
void run_sw_irr_flag(const LevelSet& S, int nl, uint8_t* flags, hipStream_t s);
void run_sw_records(const Geom& g, const Box& b, const uint8_t* labels, const int32_t* nodes,
                    int64_t nirr, int bc, double beta_plus, double beta_minus, double* rec64,
                    float* rec32, int32_t* irr_index, hipStream_t s);
// dense scaled SW matrix on the coarsest level (rows/cols = listed unknowns), then its inverse
void run_coarse_assemble(const Box& b, int dim, int periodic, const uint8_t* labels, const int32_t* irr_index,
                         const double* rec64, const int32_t* list, const int32_t* col_of, int64_t nc,
                         double* A, hipStream_t s);
void run_coarse_invert(double* A, double* Ainv, int64_t nc, int* d_err, hipStream_t s);
void run_fill_int(int32_t* p, int64_t n, int32_t v, hipStream_t s);

// ---- least squares (lsq.hip) -------------------------------------------------
struct LSParams {
    int dim, order_k, w, nrows;  // rows: w ghosts, then d/dn, then d/dx_d (gradient fits, w = 0)
    int nsides;
    double a0, b0;               // initial semi-axes (units of h)
    int max_grow;
    int mcap;                    // capacity of the per-wave scratch (rows)
};
// entries per fit of the staging layout of pass 0 (64 lanes x rows per lane)
int ls_segment(int dim);
// 3D (4,5) fits in staging layout by the corrected semi-normal equations (set
// search, moments, Cholesky + solve, rows, solve, rows); mom (then L), zc,
// rho: ls3_csne_doubles_per_fit() doubles per fit between them, zc and rho
// 140 each
void run_ls3_csne(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp, const LSParams& P,
                  int32_t* m_out, int32_t* grow_out, int32_t* st_idx, double* S, double* Sc, uint8_t* route,
                  double* mom, double* zc, double* rho, int* d_err, hipStream_t s);
int64_t ls3_csne_doubles_per_fit();
// staging -> CSR for the register-path fits (route[cs] == 0)
void run_ls_compact(int64_t ncs, int seg, int nrows, const int32_t* m, const uint8_t* route, const int64_t* ptr,
                    const int32_t* st_idx, const double* st_S, int32_t* idx, double* S, hipStream_t s);
// pass 0 with idx/S/Sc set (register path only) also writes the weights in the
// staging layout (segments of ls_segment(dim) entries); pass 1 writes CSR.
// pass 0: sizes (m, growth) per control point side; pass 1: fill idx / weights.
// cs_list == nullptr: all fits by the register path (oversized ones flagged in route);
// otherwise only the listed fits, with the global scratch (scratch_waves slabs).
void run_ls(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp, const LSParams& P,
            int pass, int32_t* m_out, int32_t* grow_out, const int64_t* ptr, int32_t* idx,
            double* S, double* Sc, double* scratch, int64_t scratch_waves, int* d_err,
            const int32_t* cs_list, int64_t n_list, uint8_t* route, hipStream_t s);

// ---- operators (ops.hip) -------------------------------------------------------
struct GhostDev {
    int bc, nsides, w, nrows;
    double beta_plus, beta_minus;
    const int64_t* ptr;   // [ncs + 1]
    const int32_t* idx;   // [nnz] local indices
    const double* W;      // [nrows][nnz] apply weights
    const double* Sc;     // [ncs][nrows] weights of u(x_c) (raw)
    const double* dcoef;  // [ncs][w] data coefficients (Dirichlet / Neumann)
    int64_t nnz, ncp;
};
void run_ghosts(const GhostDev& G, const double* x, const double* cpdata, int with_data, double* ghost,
                hipStream_t s);
// the same on a periodic grid whose storage box is the periodic cell (n nodes
// per axis, neighbours modulo n), (4,5) scheme: in 2D one thread per node; in 3D
// the z-march with wrapped loads (part 1) and the listed irregular nodes (part 2)
void run_ho_apply_periodic(int dim, const Box& b, int n, const uint8_t* labels, const int32_t* irr_index,
                           const int32_t* slots, const int32_t* irr_nodes, int64_t nirr, const double* ghost,
                           double inv_h2, double beta_plus, double beta_minus, const double* x, double* y,
                           hipStream_t s, int part = 0);
// part: 0 = the whole apply, 1 = the stencil kernel alone, 2 = the 3D irregular-node kernel alone
void run_ho_apply(int dim, const Box& b, const int* core_lo, const int* core_hi, const uint8_t* labels,
                  const int32_t* irr_index, const int32_t* slots, const int32_t* irr_nodes, int64_t nirr,
                  const double* ghost, const double* boxval, int w, double inv_h2, double beta_plus,
                  double beta_minus, const double* x, double* y, int with_data, hipStream_t s, int part = 0);

// V-cycle kernels; T = arithmetic type, S = iterate storage type
struct LevelDev {
    int dim, n;
    Box box;
    int core_lo[3], core_hi[3];
    const uint8_t* labels;
    const int32_t* irr_index;
    const double* rec64;
    const float* rec32;
    // Layout of the level's z and b.  split = 0: the storage box, x fastest.
    // split = 1 (3D grid levels): two colour arrays of `half` entries each; node
    // (i, j, k) of colour c = (i + j + k) & 1 sits at c * half + r * hx + (a >> 1),
    // r = (j - lo_y) + dims_y (k - lo_z) its box row and a = i - lo_x; hx is
    // (dims_x + 1) / 2 rounded up to a multiple of 4 (16-byte aligned rows of
    // four entries).  lab_split holds the labels in the same layout (0 at
    // entries of no node).
    int split, hx;
    int64_t half;
    const uint8_t* lab_split;
    // 1: periodic level whose storage box is the periodic cell (0..n-1 per
    // axis); neighbours are taken modulo n (box layout only)
    int periodic;
};
// entries of a level vector and the index of node (i, j, k) in it
__host__ __device__ inline int64_t vsize(const LevelDev& L) { return L.split ? 2 * L.half : L.box.size(); }
__host__ __device__ inline int64_t vidx(const LevelDev& L, int i, int j, int k) {
    if (!L.split) return L.box.idx(i, j, k);
    const int64_t r = (int64_t)(j - L.box.lo[1]) + (int64_t)L.box.dims[1] * (k - L.box.lo[2]);
    return (int64_t)((i + j + k) & 1) * L.half + r * L.hx + ((i - L.box.lo[0]) >> 1);
}
template <typename T, typename S>
void run_rbgs(const LevelDev& L, int colour, S* z, const T* b, hipStream_t s);
template <typename T, typename S>
void run_resid_restrict(const LevelDev& F, const LevelDev& C, const S* z, const T* b, T* bc, hipStream_t s,
                        S* zc0 = nullptr);  // zc0 (3D): also the coarse iterate after its first half-sweep from zero
template <typename T, typename S>
void run_prolong(const LevelDev& F, const LevelDev& C, int mode, const S* zc, S* z, hipStream_t s);
template <typename T, typename S>
void run_sw_apply(const LevelDev& L, const S* z, T* y, hipStream_t s);
template <typename T, typename S>
void run_coarse_solve(const LevelDev& L, const int32_t* list, int64_t nc, const T* Ainv, const T* b, S* z,
                      hipStream_t s);
template <typename S>
void run_zero(S* p, int64_t n, hipStream_t s);
// level-vector layout conversions (identity copies for split = 0)
template <typename U>
void run_box_to_level(const LevelDev& L, const U* boxed, U* lev, hipStream_t s);
template <typename U>
void run_level_to_box(const LevelDev& L, const U* lev, U* boxed, hipStream_t s);

// the levels first..last of a V-cycle (last = coarsest) in one workgroup
struct TailDev {
    int first, last, mode, nu_pre, nu_post;
    int64_t nc;
    const int32_t* clist;
    const void* Ainv;
    LevelDev lev[MAX_LEVELS];
    void* z[MAX_LEVELS];
    void* b[MAX_LEVELS];
    int64_t lds_z[MAX_LEVELS], lds_b[MAX_LEVELS];  // byte offsets of the LDS copies
};
// dynamic LDS the LDS-resident tail may request
constexpr int64_t TAIL_LDS_MAX = 144 * 1024;
// lds_bytes > 0: the LDS-resident tail with that much dynamic LDS (layout in
// TailDev::lds_z / lds_b); 0: the tail on global memory
template <typename T, typename S>
void run_tail(int dim, const TailDev* d_tail, int64_t lds_bytes, hipStream_t s);
void enable_tail_lds();
// the tails of up to TAIL_BATCH_MAX independent problems (same precision and
// dimension) in one launch, one workgroup each; lds[q] as run_tail's lds_bytes
constexpr int TAIL_BATCH_MAX = 64;
struct TailBatch {
    int count;
    const TailDev* d[TAIL_BATCH_MAX];
    int64_t lds[TAIL_BATCH_MAX];
};
template <typename T, typename S>
void run_tail_batch(int dim, const TailBatch& B, hipStream_t s);
// fused legs (2D): zero + nu sweeps + residual + half-weighting; prolongation + nu sweeps.
// Return false when the fused form does not apply (the caller launches the unfused kernels).
// cast: the down leg also makes b from the FP64 input v (as run_cast_in, b is then
// written); out: the up leg writes the FP64 output (as run_cast_out, on the core
// only) instead of z_out.
struct CastInArgs {
    const double* v;
    const double* scale;  // device: 1 / max |v|
    double h2, bp, bm;
};
template <typename T, typename S>
bool run_down_fused(const LevelDev& F, const LevelDev& C, const T* b, S* z, T* bc, int nu, hipStream_t s,
                    const CastInArgs* cast = nullptr);
template <typename T, typename S>
bool run_up_fused(const LevelDev& F, const LevelDev& C, int mode, const S* zc, const T* b, const S* z_in, S* z_out,
                  int nu, hipStream_t s, double* out = nullptr, const double* out_scale = nullptr);

// casts at the precision boundary: rhs0 = scale * h2 * v / beta(node); v FP64, level-0 box
template <typename T>
void run_cast_in(const LevelDev& L, const double* v, const double* scale_dev, double h2, double beta_plus,
                 double beta_minus, T* rhs, hipStream_t s);
template <typename S>
void run_cast_out(const LevelDev& L, const S* z, const double* scale_dev, double* out, hipStream_t s);
// colour-split 3D level 0: run_cast_in + zero iterate + the colour-0 half-sweep in one pass
template <typename T, typename S>
void run_cast_sweep0(const LevelDev& L, const double* v, const double* scale_dev, double h2, double bp, double bm,
                     T* b, S* z, hipStream_t s);
// colour-split 3D level 0: the colour-1 half-sweep + run_cast_out in one pass (out zero off the core rows)
template <typename T, typename S>
void run_rbgs_out(const LevelDev& L, const S* z, const T* b, double* out, const double* scale_dev, hipStream_t s);

// apply weights from the raw stencils (Neumann closure folded in) and data coefficients
void run_apply_weights(int bc, const int64_t* ptr, int64_t ncs, int w, int nrows, const double* S, const double* Sc,
                       double beta, int64_t nnz, double* W, double* dcoef, hipStream_t s);
// b[i] = scale * a[i] with conversion between double, float and half
template <typename A, typename B>
void run_convert(const A* a, B* b, int64_t n, double scale, hipStream_t s);

// ---- post-processing of a solution (Sec. 2.4) -------------------------------------
// grad[d * (n+1)^dim + f] = d/dx_d u at every unknown f (order-2w central first
// derivative over the extended function; ghost values of x must be current)
void run_ho_gradient(int dim, const Box& b, const int* core_lo, const int* core_hi, int n, const uint8_t* labels,
                     const int32_t* irr_index, const int32_t* slots, const double* ghost, const double* boxval, int w,
                     double inv_h, const double* x, double* grad, hipStream_t s);
struct BQDev {
    int bc, nsides, w, nrows;      // nrows: rows of the fits (w ghosts + the normal derivative)
    double beta_plus, beta_minus;
    const int64_t* ptr;            // [ncs + 1]
    const int32_t* idx;            // [nnz] storage-box indices
    const double* Sd;              // [nnz] the normal-derivative row of the fits
    const double* Sc;              // [ncs][nrows] weights of u(x_c)
    int64_t ncp;
};
// q[c]: du/dn (Dirichlet), u (Neumann) or du+/dn (interface) at control point c
void run_boundary_quantity(const BQDev& B, const double* x, const double* cpdata, double* q, hipStream_t s);
// Gradient of the solved side's fit at every control point from the gradient
// fits (rows: d/dn, then d/dx_d), and optionally the wall velocity's pressure
// coefficient C_p = 1 - |grad + U|^2 / |U|^2 for a free stream U.
struct WGDev {
    int bc, nsides, dim;           // fit rows: 1 + dim
    double beta_plus, beta_minus;
    const int64_t* ptr;            // [ncs + 1]
    const int32_t* idx;            // [nnz] storage-box indices
    const double* S;               // [1 + dim][nnz]
    const double* Sc;              // [ncs][1 + dim] weights of u(x_c)
    int64_t ncp;
    double u_inf[3];               // free stream (C_p only)
};
void run_wall_gradient(const WGDev& G, const double* x, const double* cpdata, double* grad, double* cp,
                       hipStream_t s);
void run_fill(double* p, int64_t n, double v, hipStream_t s);

// full grid <-> storage box
void run_full_to_box(int dim, int n, const Box& b, const double* full, double* boxed, const uint8_t* labels,
                     int only_unknowns, hipStream_t s);
void run_box_to_full(int dim, int n, const Box& b, const double* boxed, const uint8_t* labels, double fill,
                     double* full, hipStream_t s);

// ---- vector kernels (blas.hip) ---------------------------------------------------
// Deterministic reductions: a fixed grid of RED_BLOCKS blocks, per-block partials
// combined in a fixed order by a one-block second stage.
constexpr int RED_BLOCKS = 1024;
constexpr int KRED = 16;  // values per reduction launch
// reduction workspace: (KRED + 1) * RED_BLOCKS partials
constexpr int64_t RED_PART_DOUBLES = (int64_t)(KRED + 1) * RED_BLOCKS;
constexpr int RED_THREADS = 256;
// out[i] = <V_i, w> for i < k; V_i = V + i * ld; out[k] = <w, w> if with_norm
void run_multidot(const double* V, int64_t ld, int k, const double* w, int64_t n, double* part, double* out,
                  hipStream_t s, double* host_out = nullptr, int with_norm = 0);
// w -= sum_{i<k} h[i] V_i; then out[i] = <V_i, w> for i < k2 and out[k2] = <w, w> (if with_norm).
// gated: h is a first Gram-Schmidt pass's record (k dots, then |w|^2) and the pass runs only when
// that pass left too little of w; otherwise w is untouched, out[0..k] = h[0..k] and host_out
// records a zero correction.  host_out[63] = 1 if the pass ran, 0 if not.
void run_update_dot(const double* V, int64_t ld, int k, const double* h, double* w, int64_t n, int k2,
                    int with_norm, double* part, double* out, hipStream_t s, double* host_out = nullptr,
                    bool gated = false);
// the streaming first stage of run_update_dot alone (block partials in part)
void run_update_dot_stage1(const double* V, int64_t ld, int k, const double* h, double* w, int64_t n, int k2,
                           int with_norm, double* part, hipStream_t s);
// y = x / sqrt(*nrm2)
void run_normalize(const double* x, const double* nrm2, double* y, int64_t n, hipStream_t s);
// y = (w - V h) / sqrt(h[k] - |h|^2) (last CGS pass + normalisation; h[k] = |w|^2);
// the squared norm to *nrm2_out, max |y| over y's first n_max entries (all n if
// n_max < 0) and its reciprocal to scale_out[0..1]
void run_update_scale(const double* V, int64_t ld, int k, const double* h, const double* w, double* y, int64_t n,
                      double* nrm2_out, double* part, double* scale_out, hipStream_t s, double* nrm2_host = nullptr,
                      int64_t n_max = -1);
// x += sum_{i<k} y[i] Z_i  (y on the device)
void run_axpy_multi(const double* Z, int64_t ld, int k, const double* y, double* x, int64_t n, hipStream_t s);
// y = a x + b y
void run_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
void run_copy(const double* x, double* y, int64_t n, hipStream_t s);
// bordered singular system: x[n] = *alpha_src; y[unknowns] += x[n]; y[n] = sum of
// x over the unknowns
void run_border(double* x, const double* alpha_src, const uint8_t* labels, int64_t n, double* y, double* part,
                hipStream_t s);
// out[0] = max |x|, out[1] = 1 / max|x| (1 if zero)
void run_absmax(const double* x, int64_t n, double* part, double* out, hipStream_t s);
// out[0] = <x, x>
void run_norm2(const double* x, int64_t n, double* part, double* out, hipStream_t s);

// ---- manufactured data (synth.hip) ------------------------------------------------
void run_synth_cp(int kind, int dim, int bc, const CPDev& cp, double beta_plus, double beta_minus, double* cpdata,
                  hipStream_t s);
// f (box, at unknowns) and box-face values from the closed-form u
void run_synth_nodes(int kind, const Geom& g, const Box& b, const uint8_t* labels, double beta_plus, double beta_minus,
                     double* f, double* boxval, hipStream_t s);
// atomically maxes the bit pattern of max |u_full - u_exact| over the unknowns into *out
void run_synth_err(int kind, const Geom& g, const Box& b, const uint8_t* labels, const double* u,
                   unsigned long long* out, hipStream_t s,
                   double shift = 0.0);
// per-block sums of u - u_exact and counts over the unknowns into part[2 * blocks];
// returns the block count (at most 2048)
int run_synth_diff_sum(int kind, const Geom& g, const Box& b, const uint8_t* labels, const double* u, double* part,
                       hipStream_t s);

}  // namespace iim
