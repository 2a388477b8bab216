// Problem state held by an iim_problem handle.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "kernels.h"

namespace iim {

void set_error(const std::string& m);
const char* last_error();

// Owner of every device allocation of a handle.  Allocations are stream
// ordered (hipMallocAsync / hipFreeAsync on the handle's stream) from the
// device's default memory pool, so that setup and teardown of one handle never
// synchronise the device while other handles are solving on other streams.
// Device memory of one handle.  Blocks come from a process-wide cache of idle
// blocks (per device) or, when none fits, from the device's stream-ordered
// pool.  A block the handle releases while alive is kept for the handle's own
// later allocations (its work is ordered on the handle's one stream); when the
// handle ends, after its stream has drained, all its blocks return to the
// process cache.  hipMallocAsync / hipFreeAsync calls cost tens to hundreds of
// microseconds each, which dominated setup and teardown of small problems.
struct DevMem {
    struct Block {
        void* p;
        size_t bytes;  // size of the block (>= the request)
    };
    std::vector<Block> blocks;  // live
    std::vector<Block> spare;   // released by this handle, reusable by it
    hipStream_t stream = nullptr;
    int device = 0;
    size_t current = 0, peak = 0;  // bytes of live blocks
    void* alloc(size_t bytes);
    void release(void* p);
    void release_all();  // drains the stream, then hands every block to the process cache
    ~DevMem();
};

// keeps freed pool memory cached in the process (set once per device)
void configure_pool(int device);
// frees the process cache of idle blocks of the current device and trims its pool
void trim_pool();

struct Problem;
// Runs the tail of a problem's V-cycle (the levels from tail_first down, coarse
// solve included) in place of the problem's own launch, for instance batched
// with the tails of other problems.  Called on the host thread that enqueues
// the problem's work; on return the tail is ordered after everything enqueued
// before on p.stream and before everything enqueued after.
struct TailRunner {
    virtual void run(Problem& p) = 0;
    virtual ~TailRunner() = default;
};

struct Level {
    int n = 0;
    double h = 0.0;
    Geom geom{};
    Box box{};
    int core_lo[3] = {0, 0, 0}, core_hi[3] = {-1, -1, -1};
    int64_t nunk = 0;
    uint8_t* labels = nullptr;
    int64_t nirr = 0;
    int32_t* irr_index = nullptr;
    double* rec64 = nullptr;
    float* rec32 = nullptr;
    void* z = nullptr;   // iterate (storage type)
    void* z2 = nullptr;  // 2D: output buffer of the fused up leg (it reads z)
    void* b = nullptr;  // right-hand side (arithmetic type)
    // layout of z, z2 and b: 0 = storage box; 1 = colour-split (3D levels
    // above the tail), hx entries per box row and colour, half per colour
    int split = 0, hx = 0;
    int64_t half = 0;
    uint8_t* lab_split = nullptr;  // labels in the colour-split layout
    int64_t vsize() const { return split ? 2 * half : box.size(); }
};

constexpr int64_t TAIL_MAX_NODES = 4096;  // levels handled by the one-workgroup tail kernel
constexpr int64_t LS_SCRATCH_WAVES = 2048;  // waves of the global-memory least-squares path
constexpr int HCOL = 3 * 64;               // doubles of one Hessenberg column record (two CGS passes + norm)
constexpr int HPIN_DOUBLES = 12 * HCOL;    // one record per inner iteration (restart <= 11)

struct Problem {
    DevMem mem;
    hipStream_t stream = nullptr;
    iim_grid grid{};
    iim_options opt{};
    int dim = 2, kind = 0, side = 0, bc = 0, nsides = 1, w = 2;
    // interior domain with a Neumann boundary: L 1 = 0, solved as the bordered
    // system [L 1; 1^T 0] [u; alpha] = [b; 0]; Krylov vectors then carry alpha
    // in entry box.size()
    bool singular = false;
    double h = 0.0;
    std::vector<double> params;
    double* d_params = nullptr;

    // level 0 storage and control points
    Box box{};
    CPDev cp{};
    // least-squares stencils: CSR over control-point sides
    std::vector<int64_t> h_ptr;
    int64_t nnz = 0;
    int nrows = 0, nrows_apply = 0;
    int64_t* ls_ptr = nullptr;
    int32_t* ls_idx = nullptr;
    double* ls_S = nullptr;   // [nrows][nnz] raw weights of the grid points
    double* ls_Sc = nullptr;  // [ncs][nrows] weights of u(x_c)
    // fits with the normal-derivative row, made on first use when the setup's
    // fits lack it (Dirichlet): same layout with w + 1 rows
    int64_t* nd_ptr = nullptr;
    int32_t* nd_idx = nullptr;
    double* nd_S = nullptr;
    double* nd_Sc = nullptr;
    int64_t nd_nnz = 0;
    // fits with the rows d/dn and d/dx_d (wall gradient), made on first use
    int64_t* gd_ptr = nullptr;
    int32_t* gd_idx = nullptr;
    double* gd_S = nullptr;
    double* gd_Sc = nullptr;
    int64_t gd_nnz = 0;
    double* W_apply = nullptr;
    double* dcoef = nullptr;
    double* ghost = nullptr;
    double* cpdata = nullptr;
    // irregular high-order nodes
    int64_t ho_nirr = 0;
    int32_t* ho_irr_index = nullptr;
    int32_t* ho_slots = nullptr;
    int32_t* ho_nodes = nullptr;  // their storage indices
    // multigrid
    std::vector<Level> levels;
    int64_t nc = 0;
    int32_t* coarse_list = nullptr;
    double* Ainv64 = nullptr;
    float* Ainv32 = nullptr;
    // solve vectors (level-0 box)
    double *boxval = nullptr, *rhs = nullptr, *xk = nullptr, *rk = nullptr, *wk = nullptr;
    double *Vb = nullptr, *Zb = nullptr;  // Krylov bases, vector i at + i * ldv
    int64_t ldv = 0;                        // box size rounded up to 64 doubles
    double *red_part = nullptr, *red_out = nullptr;
    double* red_scale = nullptr;
    hipEvent_t ev[8] = {};
    bool own_stream = false;
    int tail_first = 0;
    int64_t tail_lds_bytes = 0;  // > 0: the tail levels run in that much LDS
    bool opt_fused = true;  // LDS-tiled fused smoothing legs where available
    bool opt_split = true;  // colour-split vectors on 3D grid levels
    TailDev* d_tail = nullptr;
    double* hpin = nullptr;  // Hessenberg column records, HCOL doubles per iteration, written by kernels
    bool own_hpin = true;
    hipGraphExec_t iter_graph[16] = {};
    hipGraphExec_t pre_graph[16] = {};  // with a tail runner: iteration parts before the tail
    TailRunner* tail_runner = nullptr;  // not owned
    hipEvent_t iter_done[2] = {};  // end of inner iteration j, alternating by parity
    double t_setup_ms = 0.0;

    void setup();
    // ghost_rows: ghost functionals before the derivative rows (-1: w)
    void fit_stencils(int nr, int* d_err, int64_t*& ptr_out, int32_t*& idx_out, double*& S_out, double*& Sc_out,
                      std::vector<int64_t>& hptr, int64_t& nz, int ghost_rows = -1);
    void ensure_normal_rows();
    void ensure_grad_rows();
    LevelSet level_set() const;
    LevelDev level_dev(int l) const;
    GhostDev ghost_dev() const;
    void apply_box(const double* x, double* y, int with_data);
    // the solver's operator: L x, bordered for a singular problem; alpha_src
    // (bordered only) is where x's alpha comes from, x + box.size() by default
    void apply_op(double* x, double* y, const double* alpha_src = nullptr);
    int64_t krylov_len() const { return box.size() + (singular ? 1 : 0); }
    template <typename T, typename S> bool down_leg(int l, const CastInArgs* cast);
    template <typename T, typename S> const S* up_leg(int l, const S* zres, double* out);
    // scaled: red_scale already holds max |v| (the fused orthogonalisation wrote it);
    // out_basis: out is zero off the core (a Krylov basis column)
    // part 0: the whole cycle; 1: down to the tail (exclusive); 2: from the
    // tail's result up (parts 1 and 2 leave the tail to the caller)
    template <typename T, typename S> void vcycle_t(const double* v, double* out, bool scaled, bool out_basis, int part);
    template <typename T, typename S> void vcycle_down(const double* v, bool scaled);
    template <typename T, typename S> void wcycle_t(const double* v, double* out, bool scaled);
    template <typename T, typename S> void wvisit(int l, bool zero_start);
    void vcycle(const double* v, double* out, bool scaled = false, bool out_basis = false, int part = 0);
    void iteration_body(int j, hipEvent_t* evs = nullptr, int part = 0);
    int solve(double* u_full, const double* x0_full, double* hist, int hist_cap, iim_stats* st);
    int level_op(int level, int op, const double* in1, double* out);
    template <typename T, typename S> void launch_kernel_t(int kernel);
    double time_kernel(int kernel, int reps);
    template <typename T, typename S> int level_op_t(int level, int op, const double* in1, double* out);
    // staging: a device buffer of (n+1)^dim doubles for the box data (nullptr:
    // one is allocated for the call)
    void set_boundary_data(const double* cp_data, const double* box_data, int mem_kind, double* staging = nullptr);
    void set_rhs(const double* f, int mem_kind);
    void synth_data(int kind);
    double synth_error(int kind, const double* u_full);
    ~Problem();
};

// validated construction with setup (stream: NULL creates a blocking stream
// owned by the problem); hpin: optional caller-owned fine-grained pinned buffer
// (hipHostMallocCoherent) of HPIN_DOUBLES doubles
std::unique_ptr<Problem> make_problem(const iim_grid* g, const iim_geometry* geo, const iim_options* opt,
                                      hipStream_t stream, double* hpin);
// rejects (IIM_E_INVALID_ARG) an interior Neumann sphere union whose interior
// is not connected: the bordered system fixes only one constant
void check_singular_connected(const iim_grid& g, const iim_geometry& geo);
// device bytes a problem will hold at its peak, from the request alone
int64_t estimate_bytes(const iim_grid& g, const iim_geometry& geo, const iim_options& opt);

}  // namespace iim
