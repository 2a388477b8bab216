// Host core of the library: problem setup on the device, the multigrid
// V-cycle driver, the FGMRES solver, and the C ABI (include/iim.h).
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "core.h"

namespace iim {

static thread_local std::string g_last_error;

void set_error(const std::string& m) { g_last_error = m; }
const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------
void configure_pool(int device) {
    static std::mutex mu;
    static bool done[64] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (device < 0 || device >= 64 || done[device]) return;
    int supported = 0;
    IIM_HIP(hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, device));
    if (!supported) throw Error(IIM_E_DEVICE, "the device has no stream-ordered memory pools");
    hipMemPool_t pool;
    IIM_HIP(hipDeviceGetDefaultMemPool(&pool, device));
    uint64_t keep = UINT64_MAX;
    IIM_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    done[device] = true;
}

// process-wide idle blocks, per device, by size
static std::mutex g_cache_mu;
static std::multimap<size_t, void*> g_cache[64];

// a cached block of `have` bytes serves a request of `want` bytes when the
// excess stays small (exact sizes recur: the same problem set up again)
static bool fits(size_t have, size_t want) { return have >= want && have - want <= want / 16 + 65536; }

static size_t cache_free_all(int dev) {
    std::multimap<size_t, void*> take;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        take.swap(g_cache[dev]);
    }
    size_t n = 0;
    for (auto& kv : take) {
        (void)hipFreeAsync(kv.second, nullptr);  // idle blocks: no pending work
        n += kv.first;
    }
    if (n) (void)hipStreamSynchronize(nullptr);  // back in the pool before anyone allocates again
    return n;
}

void trim_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    cache_free_all(dev);
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
}

// Library-owned streams and pinned Hessenberg buffers of ended handles, kept
// for later handles (creating either costs about a tenth of a millisecond).
static std::mutex g_res_mu;
static std::vector<std::pair<int, hipStream_t>> g_streams;
static std::vector<double*> g_hpins;

static hipStream_t take_stream(int dev) {
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        for (size_t i = 0; i < g_streams.size(); ++i)
            if (g_streams[i].first == dev) {
                hipStream_t s = g_streams[i].second;
                g_streams.erase(g_streams.begin() + i);
                return s;
            }
    }
    // a blocking stream: ordered with the legacy default stream, and capturable
    hipStream_t s = nullptr;
    IIM_HIP(hipStreamCreate(&s));
    return s;
}

static void give_stream(int dev, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_res_mu);
    g_streams.push_back({dev, s});
}

static double* take_hpin() {
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        if (!g_hpins.empty()) {
            double* p = g_hpins.back();
            g_hpins.pop_back();
            return p;
        }
    }
    double* p = nullptr;
    // fine-grained: kernels write the Hessenberg records into it directly
    IIM_HIP(hipHostMalloc((void**)&p, HPIN_DOUBLES * sizeof(double), hipHostMallocCoherent));
    return p;
}

static void give_hpin(double* p) {
    std::lock_guard<std::mutex> lk(g_res_mu);
    g_hpins.push_back(p);
}

void* DevMem::alloc(size_t bytes) {
    bytes = (std::max<size_t>(bytes, 8) + 255) / 256 * 256;
    void* p = nullptr;
    size_t got = 0;
    // the handle's own released blocks first, then the process cache (best fit)
    size_t best = SIZE_MAX;
    for (size_t i = 0; i < spare.size(); ++i)
        if (fits(spare[i].bytes, bytes) && (best == SIZE_MAX || spare[i].bytes < spare[best].bytes)) best = i;
    if (best != SIZE_MAX) {
        p = spare[best].p;
        got = spare[best].bytes;
        spare.erase(spare.begin() + best);
    } else if (device >= 0 && device < 64) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache[device].lower_bound(bytes);
        if (it != g_cache[device].end() && fits(it->first, bytes)) {
            p = it->second;
            got = it->first;
            g_cache[device].erase(it);
        }
    }
    if (!p) {
        hipError_t e = hipMallocAsync(&p, bytes, stream);
        if (e == hipErrorOutOfMemory && device >= 0 && device < 64 && cache_free_all(device) > 0) {
            (void)hipGetLastError();
            e = hipMallocAsync(&p, bytes, stream);  // idle cached blocks returned to the device first
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(e == hipErrorOutOfMemory ? IIM_E_BUDGET : IIM_E_DEVICE,
                        std::string("hipMallocAsync(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
        }
        got = bytes;
    }
    blocks.push_back({p, got});
    current += got;
    peak = std::max(peak, current);
    return p;
}

void DevMem::release(void* p) {
    for (size_t i = 0; i < blocks.size(); ++i)
        if (blocks[i].p == p) {
            current -= blocks[i].bytes;
            spare.push_back(blocks[i]);
            blocks.erase(blocks.begin() + i);
            return;
        }
}

void DevMem::release_all() {
    if (blocks.empty() && spare.empty()) return;
    if (stream) (void)hipStreamSynchronize(stream);
    if (device >= 0 && device < 64) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (auto& q : blocks) g_cache[device].emplace(q.bytes, q.p);
        for (auto& q : spare) g_cache[device].emplace(q.bytes, q.p);
    } else {
        for (auto& q : blocks) (void)hipFreeAsync(q.p, stream);
        for (auto& q : spare) (void)hipFreeAsync(q.p, stream);
    }
    blocks.clear();
    spare.clear();
    current = 0;
}

DevMem::~DevMem() { release_all(); }

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
static Box make_box(int dim, const int* mn, const int* mx, int pad, bool empty) {
    Box b;
    for (int d = 0; d < 3; ++d) {
        if (d >= dim) {
            b.lo[d] = 0;
            b.dims[d] = 1;
        } else if (empty) {
            b.lo[d] = 0;
            b.dims[d] = 1;
        } else {
            b.lo[d] = mn[d] - pad;
            b.dims[d] = mx[d] - mn[d] + 1 + 2 * pad;
        }
    }
    return b;
}

// Throws if any error bit is set in the host copy of the device error word.
static void raise_setup_error(int h, const char* what) {
    if (!h) return;
    std::string m = std::string(what) + " failed (code " + std::to_string(h) + ")";
    if (h & 2) m += ": |kappa h| >= 1/4 at a control point";
    if (h & (4 | 8)) m += ": irregular node without its crossing";
    if (h & 32) m += ": least-squares set exceeds its capacity";
    if (h & 128) m += ": least-squares fit rank deficient after growth";
    if (h & 16) m += ": singular coarse-level matrix";
    throw Error(IIM_E_GEOMETRY_UNRESOLVED, m);
}

// Least-squares fits of every control point and side with nr rows (the w ghost
// functionals, then the normal derivative at x_c when nr = w + 1): sizes and
// growth on the register path, oversized sets on the global-memory path, then
// the weights, compacted.  Outputs: ptr_out [ncs + 1], idx_out [nnz], S_out
// [nr][nnz], Sc_out [ncs][nr] and the host copy of the pointers; d_err: the
// device error word.  The pass is deterministic: a second call returns the
// same sets.
void Problem::fit_stencils(int nr, int* d_err, int64_t*& ptr_out, int32_t*& idx_out, double*& S_out,
                           double*& Sc_out, std::vector<int64_t>& hptr, int64_t& nz, int ghost_rows) {
    const Level& L0 = levels[0];
    const int64_t ncs = cp.ncp * nsides;
    int err_bits = 0;
    auto read_err = [&]() {
        IIM_HIP(hipMemcpyAsync(&err_bits, d_err, sizeof(int), hipMemcpyDeviceToHost, stream));
        IIM_HIP(hipStreamSynchronize(stream));
    };
    LSParams P;
    P.dim = dim;
    P.order_k = opt.order_k;
    P.w = ghost_rows < 0 ? w : ghost_rows;
    P.nrows = nr;
    P.nsides = nsides;
    P.a0 = opt.ls_axis_t > 0 ? opt.ls_axis_t : (double)opt.order_k;
    P.b0 = opt.ls_axis_n > 0 ? opt.ls_axis_n : opt.order_k - 0.5;
    P.max_grow = 6;
    P.mcap = dim == 2 ? 192 : 768;
    const int K = opt.order_k;
    const int p = dim == 2 ? K * (K + 1) / 2 : K * (K + 1) * (K + 2) / 6;
    const int64_t ncs1 = std::max<int64_t>(ncs, 1);
    int32_t* d_mg = (int32_t*)mem.alloc(2 * ncs1 * sizeof(int32_t));  // sizes, then growth
    int32_t* d_m = d_mg;
    int32_t* d_grow = d_mg + ncs1;
    uint8_t* d_route = (uint8_t*)mem.alloc(ncs1);
    IIM_HIP(hipMemsetAsync(d_route, 0, ncs1, stream));
    // one pass over the register path: sizes, growth and the weights, the
    // weights into fixed segments of a staging area (compacted below)
    const int seg = ls_segment(dim);
    int32_t* st_idx = (int32_t*)mem.alloc(ncs1 * seg * sizeof(int32_t));
    double* st_S = (double*)mem.alloc((size_t)nr * ncs1 * seg * sizeof(double));
    Sc_out = (double*)mem.alloc(ncs1 * nr * sizeof(double));
    if (dim == 3 && opt.order_k == 5 && nr <= 4) {  // the CSNE passes carry up to four functionals
        const int64_t per = ls3_csne_doubles_per_fit();
        double* work = (double*)mem.alloc((size_t)ncs1 * per * sizeof(double));
        run_ls3_csne(L0.geom, box, L0.labels, cp, P, d_m, d_grow, st_idx, st_S, Sc_out, d_route, work,
                     work + ncs1 * (per - 280), work + ncs1 * (per - 140), d_err, stream);
        mem.release(work);
    } else {
        run_ls(L0.geom, box, L0.labels, cp, P, 0, d_m, d_grow, nullptr, st_idx, st_S, Sc_out, nullptr, 0, d_err,
               nullptr, 0, d_route, stream);
    }
    std::vector<int32_t> hmg(2 * ncs1);
    IIM_HIP(hipMemcpyAsync(hmg.data(), d_mg, 2 * ncs1 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    read_err();
    raise_setup_error(err_bits, "control points and least-squares sizes");
    std::vector<int32_t> big;
    for (int64_t i = 0; i < ncs; ++i)
        if (hmg[ncs1 + i] == -3) big.push_back((int32_t)i);
    int32_t* d_list = nullptr;
    double* scratch = nullptr;
    int64_t waves = 0;
    if (!big.empty()) {  // oversized sets: Householder on a per-wave global scratch slab
        // each wave works through its fits one global-memory round trip at a
        // time: eight waves per CU hide those latencies (3D degree-6 fits,
        // all on this path, take 1.1 GB of slabs)
        waves = std::min<int64_t>((int64_t)big.size(), LS_SCRATCH_WAVES);
        scratch = (double*)mem.alloc((size_t)waves * (p + 4) * P.mcap * sizeof(double));
        d_list = (int32_t*)mem.alloc(big.size() * sizeof(int32_t));
        IIM_HIP(hipMemcpyAsync(d_list, big.data(), big.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        run_ls(L0.geom, box, L0.labels, cp, P, 0, d_m, d_grow, nullptr, nullptr, nullptr, nullptr, scratch, waves,
               d_err, d_list, (int64_t)big.size(), d_route, stream);
        IIM_HIP(hipMemcpyAsync(hmg.data(), d_mg, ncs1 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        read_err();
        raise_setup_error(err_bits, "least-squares sizes (large sets)");
    }
    hptr.assign(ncs + 1, 0);
    for (int64_t i = 0; i < ncs; ++i) hptr[i + 1] = hptr[i] + hmg[i];
    nz = hptr[ncs];
    ptr_out = (int64_t*)mem.alloc((ncs + 1) * sizeof(int64_t));
    IIM_HIP(hipMemcpyAsync(ptr_out, hptr.data(), (ncs + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    idx_out = (int32_t*)mem.alloc(std::max<int64_t>(nz, 1) * sizeof(int32_t));
    S_out = (double*)mem.alloc(std::max<int64_t>(nr * nz, 1) * sizeof(double));
    run_ls_compact(ncs, seg, nr, d_m, d_route, ptr_out, st_idx, st_S, idx_out, S_out, stream);
    mem.release(st_idx);
    mem.release(st_S);
    if (!big.empty())
        run_ls(L0.geom, box, L0.labels, cp, P, 1, d_m, d_grow, ptr_out, idx_out, S_out, Sc_out, scratch, waves, d_err,
               d_list, (int64_t)big.size(), d_route, stream);
    if (scratch) mem.release(scratch);
    if (d_list) mem.release(d_list);
    mem.release(d_mg);
    mem.release(d_route);
}

// Setup on the device.  The stages are batched so that the host waits for the
// device only where a size or an error decides what comes next (six waits):
// level bounding boxes; control-point counts; least-squares set sizes;
// irregular-node counts of every level; the coarsest level's rows; the end.
// The normal-derivative row of every fit for problems whose setup fitted only
// the ghost rows (Dirichlet): the fits once more with w + 1 rows, kept for
// later calls.  The sets are those of the setup (the pass is deterministic).
void Problem::ensure_normal_rows() {
    if (nrows == w + 1 || nd_S) return;
    int* d_err = (int*)mem.alloc(sizeof(int64_t));
    IIM_HIP(hipMemsetAsync(d_err, 0, sizeof(int64_t), stream));
    std::vector<int64_t> hp;
    fit_stencils(w + 1, d_err, nd_ptr, nd_idx, nd_S, nd_Sc, hp, nd_nnz);
    int err = 0;
    IIM_HIP(hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, stream));
    IIM_HIP(hipStreamSynchronize(stream));
    mem.release(d_err);
    raise_setup_error(err, "least-squares fits with the normal-derivative row");
    if (hp != h_ptr) throw Error(IIM_E_INTERNAL, "normal-derivative fits: the sets differ from the setup's");
}

// The gradient fits of the wall derivatives: every control point fitted once
// more with the rows d/dn and d/dx_d (no ghost rows), kept for later calls.
// The sets are those of the setup (the pass is deterministic).
void Problem::ensure_grad_rows() {
    if (gd_S) return;
    int* d_err = (int*)mem.alloc(sizeof(int64_t));
    IIM_HIP(hipMemsetAsync(d_err, 0, sizeof(int64_t), stream));
    std::vector<int64_t> hp;
    fit_stencils(1 + dim, d_err, gd_ptr, gd_idx, gd_S, gd_Sc, hp, gd_nnz, 0);
    int err = 0;
    IIM_HIP(hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, stream));
    IIM_HIP(hipStreamSynchronize(stream));
    mem.release(d_err);
    raise_setup_error(err, "least-squares fits with the derivative rows");
    if (hp != h_ptr) throw Error(IIM_E_INTERNAL, "gradient fits: the sets differ from the setup's");
}

void Problem::setup() {
    const double t0 = now_ms();
    w = opt.order_n / 2;
    h = (grid.hi - grid.lo) / grid.n;
    nsides = (side == IIM_SIDE_INTERFACE) ? 2 : 1;
    // small device scalars: [0] error bits, [1..] counts written by selections
    constexpr int NSC = 64;
    int64_t* d_sc = (int64_t*)mem.alloc(NSC * sizeof(int64_t));
    IIM_HIP(hipMemsetAsync(d_sc, 0, NSC * sizeof(int64_t), stream));
    int* d_err = (int*)d_sc;
    int64_t h_sc[NSC];
    auto read_sc = [&](int count) {
        IIM_HIP(hipMemcpyAsync(h_sc, d_sc, count * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        IIM_HIP(hipStreamSynchronize(stream));
    };
    auto err_bits = [&]() { return (int)(h_sc[0] & 0xffffffff); };
    d_params = (double*)mem.alloc(params.size() * sizeof(double));
    IIM_HIP(hipMemcpyAsync(d_params, params.data(), params.size() * sizeof(double), hipMemcpyHostToDevice, stream));

    // ---- levels: bounding boxes of the unknowns of every level at once  [wait 1]
    std::vector<int> sizes{grid.n};
    while (sizes.back() > opt.coarsest_n) sizes.push_back((sizes.back() + 1) / 2);
    const int nl = (int)sizes.size();
    if (nl > MAX_LEVELS || nl + 8 > NSC) throw Error(IIM_E_INVALID_ARG, "too many multigrid levels");
    levels.resize(nl);
    {
        std::vector<int> h_bb(8 * nl);
        int* d_bb = (int*)mem.alloc(8 * nl * sizeof(int));
        unsigned long long* d_cnt = (unsigned long long*)mem.alloc(nl * sizeof(unsigned long long));
        int* d_part = (int*)mem.alloc(classify_part_ints(nl) * sizeof(int));
        GeomSet G{};
        for (int l = 0; l < nl; ++l) {
            Level& L = levels[l];
            L.n = sizes[l];
            L.h = h * (double)(1 << l);
            L.geom = Geom{kind, side, dim, L.n, grid.lo, L.h, d_params, grid.periodic ? 1 : 0};
            G.g[l] = L.geom;
        }
        run_classify_levels(G, nl, d_part, d_bb, d_cnt, stream);
        std::vector<unsigned long long> h_cnt(nl);
        IIM_HIP(hipMemcpyAsync(h_bb.data(), d_bb, 8 * nl * sizeof(int), hipMemcpyDeviceToHost, stream));
        IIM_HIP(hipMemcpyAsync(h_cnt.data(), d_cnt, nl * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
        IIM_HIP(hipStreamSynchronize(stream));
        mem.release(d_bb);
        mem.release(d_cnt);
        mem.release(d_part);
        for (int l = 0; l < nl; ++l) {
            Level& L = levels[l];
            const int* bb = h_bb.data() + 8 * l;
            if (bb[6] && !grid.periodic)
                throw Error(IIM_E_GEOMETRY_UNRESOLVED, "the immersed body touches the domain box");
            L.nunk = (int64_t)h_cnt[l];
            const bool empty = h_cnt[l] == 0;
            if (grid.periodic) {
                // the storage box is the periodic cell: nodes 0..n-1 on every axis
                // (neighbours are taken modulo n), no padding
                L.box = Box{{0, 0, 0}, {L.n, L.n, dim == 3 ? L.n : 1}};
                for (int d = 0; d < 3; ++d) {
                    L.core_lo[d] = 0;
                    L.core_hi[d] = d < dim ? L.n - 1 : 0;
                }
            } else {
                int mn[3] = {bb[0], bb[1], dim == 3 ? bb[2] : 0};
                int mx[3] = {bb[3], bb[4], dim == 3 ? bb[5] : 0};
                L.box = make_box(dim, mn, mx, l == 0 ? w : 1, empty);  // level 0: the stencil's reach
                for (int d = 0; d < 3; ++d) {
                    L.core_lo[d] = empty ? 1 : (d < dim ? mn[d] : 0);
                    L.core_hi[d] = empty ? 0 : (d < dim ? mx[d] : 0);
                }
            }
            if (L.box.size() > (int64_t)INT32_MAX) throw Error(IIM_E_BUDGET, "storage box exceeds 2^31 nodes");
            L.labels = (uint8_t*)mem.alloc(L.box.size());
        }
        run_box_labels(level_set(), nl, stream);
    }
    Level& L0 = levels[0];
    if (L0.nunk == 0) throw Error(IIM_E_INVALID_ARG, "the problem has no unknowns");
    box = L0.box;
    // scratch of the flagged-node selections (stream ordered)
    int* sel_part = (int*)mem.alloc(SEL_BLOCKS * SEL_MAX * sizeof(int));

    // ---- control points (level 0): crossings of each axis  [wait 2]
    {
        uint8_t* flags = (uint8_t*)mem.alloc(dim * box.size());
        run_cp_flags(L0.geom, box, L0.labels, flags, stream);
        std::vector<int32_t*> per_axis(dim);
        SelItem items[3];
        for (int a = 0; a < dim; ++a) {
            per_axis[a] = (int32_t*)mem.alloc(box.size() * sizeof(int32_t));
            items[a] = SelItem{flags + a * box.size(), box.size(), per_axis[a], d_sc + 1 + a};
        }
        select_flagged_multi(items, dim, sel_part, stream);
        mem.release(flags);
        read_sc(1 + dim);
        int64_t ncp = 0;
        cp.axis_start[0] = 0;
        for (int a = 0; a < 3; ++a) {
            if (a < dim) ncp += h_sc[1 + a];
            cp.axis_start[a + 1] = (int)ncp;
        }
        cp.ncp = ncp;
        cp.nsides = nsides;
        cp.lower = (int32_t*)mem.alloc(std::max<int64_t>(ncp, 1) * sizeof(int32_t));
        cp.axis = (int32_t*)mem.alloc(std::max<int64_t>(ncp, 1) * sizeof(int32_t));
        cp.a = (int32_t*)mem.alloc(std::max<int64_t>(ncp, 1) * nsides * sizeof(int32_t));
        cp.dir = (int32_t*)mem.alloc(std::max<int64_t>(ncp, 1) * nsides * sizeof(int32_t));
        cp.x = (double*)mem.alloc(3 * std::max<int64_t>(ncp, 1) * sizeof(double));
        cp.n = (double*)mem.alloc(3 * std::max<int64_t>(ncp, 1) * sizeof(double));
        cp.kappa = (double*)mem.alloc(std::max<int64_t>(ncp, 1) * sizeof(double));
        for (int a = 0; a < dim; ++a) {
            const int64_t c = h_sc[1 + a];
            if (c) {
                IIM_HIP(hipMemcpyAsync(cp.lower + cp.axis_start[a], per_axis[a], c * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, stream));
                run_fill_int(cp.axis + cp.axis_start[a], c, a, stream);
            }
            mem.release(per_axis[a]);
        }
        run_cp_compute(L0.geom, box, L0.labels, cp, d_err, stream);
    }

    // ---- least-squares stencils (FP64): sizes  [wait 3], then the fits
    const int64_t ncs = cp.ncp * nsides;
    // rows: the w ghost functionals, then the normal derivative at x_c, which the
    // Neumann and interface closures use; Dirichlet problems fit it only when the
    // boundary-quantity post-processing first asks (fit_stencils once more)
    nrows = w + ((bc == IIM_BC_DIRICHLET) ? 0 : 1);
    {
        fit_stencils(nrows, d_err, ls_ptr, ls_idx, ls_S, ls_Sc, h_ptr, nnz);
        const int64_t ncs1 = std::max<int64_t>(ncs, 1);
        // apply weights
        dcoef = (double*)mem.alloc(ncs1 * w * sizeof(double));
        if (bc == IIM_BC_NEUMANN) {
            W_apply = (double*)mem.alloc(std::max<int64_t>(w * nnz, 1) * sizeof(double));
            nrows_apply = w;
        } else {
            W_apply = ls_S;
            nrows_apply = nrows;
        }
        run_apply_weights(bc, ls_ptr, ncs, w, nrows, ls_S, ls_Sc, opt.beta_plus, nnz,
                          bc == IIM_BC_NEUMANN ? W_apply : nullptr, dcoef, stream);
        ghost = (double*)mem.alloc(ncs1 * w * sizeof(double));
        cpdata = (double*)mem.alloc(std::max<int64_t>(cp.ncp, 1) * 2 * sizeof(double));
        IIM_HIP(hipMemsetAsync(cpdata, 0, std::max<int64_t>(cp.ncp, 1) * 2 * sizeof(double), stream));
    }

    // ---- irregular nodes: high-order (level 0) and Shortley-Weller (every level),
    // selected together  [wait 4]
    std::vector<int32_t*> sw_sel(nl);
    int32_t* ho_sel = (int32_t*)mem.alloc(box.size() * sizeof(int32_t));
    {
        LevelSet S = level_set();
        int64_t nflags = box.size();  // high-order flags first, then each level's SW flags
        for (int l = 0; l < nl; ++l) {
            S.off[l] = nflags;
            nflags += levels[l].box.size();
        }
        uint8_t* flags = (uint8_t*)mem.alloc(nflags);
        run_ho_irr_flag(L0.geom, box, L0.labels, flags, w, stream);
        run_sw_irr_flag(S, nl, flags, stream);
        std::vector<SelItem> items;
        items.push_back(SelItem{flags, box.size(), ho_sel, d_sc + 4});
        for (int l = 0; l < nl; ++l) {
            sw_sel[l] = (int32_t*)mem.alloc(levels[l].box.size() * sizeof(int32_t));
            items.push_back(SelItem{flags + S.off[l], levels[l].box.size(), sw_sel[l], d_sc + 8 + l});
        }
        select_flagged_multi(items.data(), (int)items.size(), sel_part, stream);
        mem.release(flags);
    }
    read_sc(8 + nl);
    raise_setup_error(err_bits(), "least-squares fits");
    mem.release(sel_part);
    {
        ho_nirr = h_sc[4];
        ho_irr_index = (int32_t*)mem.alloc(box.size() * sizeof(int32_t));
        run_fill_int(ho_irr_index, box.size(), -1, stream);
        ho_slots = (int32_t*)mem.alloc(std::max<int64_t>(ho_nirr, 1) * 2 * dim * sizeof(int32_t));
        run_ho_irr_records(L0.geom, box, L0.labels, cp, ho_sel, ho_nirr, ho_slots, ho_irr_index, w, d_err, stream);
        ho_nodes = (int32_t*)mem.alloc(std::max<int64_t>(ho_nirr, 1) * sizeof(int32_t));
        if (ho_nirr)
            IIM_HIP(hipMemcpyAsync(ho_nodes, ho_sel, ho_nirr * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
        mem.release(ho_sel);
    }
    const int R = 1 + 2 * dim;
    for (int l = 0; l < nl; ++l) {
        Level& L = levels[l];
        const int64_t bs = L.box.size();
        L.nirr = h_sc[8 + l];
        L.irr_index = (int32_t*)mem.alloc(bs * sizeof(int32_t));
        run_fill_int(L.irr_index, bs, -1, stream);
        L.rec64 = (double*)mem.alloc(std::max<int64_t>(L.nirr, 1) * R * sizeof(double));
        L.rec32 = (float*)mem.alloc(std::max<int64_t>(L.nirr, 1) * R * sizeof(float));
        run_sw_records(L.geom, L.box, L.labels, sw_sel[l], L.nirr, bc, opt.beta_plus, opt.beta_minus, L.rec64,
                       L.rec32, L.irr_index, stream);
        mem.release(sw_sel[l]);
    }

    // ---- coarsest level: dense inverse of the scaled SW matrix  [wait 5]
    {
        Level& Lc = levels.back();
        int64_t bs = Lc.box.size();
        std::vector<uint8_t> lab(bs);
        std::vector<int32_t> irr(bs);
        std::vector<double> rec(std::max<int64_t>(Lc.nirr, 1) * R);
        IIM_HIP(hipMemcpyAsync(lab.data(), Lc.labels, bs, hipMemcpyDeviceToHost, stream));
        IIM_HIP(hipMemcpyAsync(irr.data(), Lc.irr_index, bs * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        IIM_HIP(hipMemcpyAsync(rec.data(), Lc.rec64, rec.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
        read_sc(1);
        raise_setup_error(err_bits(), "irregular records");
        std::vector<int32_t> list, col_of(bs, -1);
        for (int64_t l = 0; l < bs; ++l) {
            if (!is_unknown(lab[l])) continue;
            double diag = (lab[l] & F_SW_IRR) ? rec[(int64_t)irr[l] * R] : -2.0 * dim;
            if (diag == 0.0) continue;
            col_of[l] = (int32_t)list.size();
            list.push_back((int32_t)l);
        }
        nc = (int64_t)list.size();
        if (nc > 4096) throw Error(IIM_E_INVALID_ARG, "coarsest level too large for a dense solve");
        coarse_list = (int32_t*)mem.alloc(std::max<int64_t>(nc, 1) * sizeof(int32_t));
        int32_t* d_col = (int32_t*)mem.alloc(bs * sizeof(int32_t));
        if (nc) IIM_HIP(hipMemcpyAsync(coarse_list, list.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        IIM_HIP(hipMemcpyAsync(d_col, col_of.data(), bs * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        double* A = (double*)mem.alloc(std::max<int64_t>(nc * nc, 1) * sizeof(double));
        Ainv64 = (double*)mem.alloc(std::max<int64_t>(nc * nc, 1) * sizeof(double));
        Ainv32 = (float*)mem.alloc(std::max<int64_t>(nc * nc, 1) * sizeof(float));
        run_coarse_assemble(Lc.box, dim, grid.periodic, Lc.labels, Lc.irr_index, Lc.rec64, coarse_list, d_col, nc, A, stream);
        if (singular && nc) {
            // the coarsest SW matrix annihilates constants as the fine operator
            // does: invert the bordered [A 1; 1^T 0] and keep its leading block,
            // which maps b to the coarse values of the bordered solution of
            // [b; 0] (they sum to zero)
            const int64_t nb = nc + 1;
            std::vector<double> Ah(nc * nc), Ab(nb * nb, 0.0);
            IIM_HIP(hipMemcpyAsync(Ah.data(), A, nc * nc * sizeof(double), hipMemcpyDeviceToHost, stream));
            IIM_HIP(hipStreamSynchronize(stream));
            for (int64_t r = 0; r < nc; ++r) {
                for (int64_t c = 0; c < nc; ++c) Ab[r * nb + c] = Ah[r * nc + c];
                Ab[r * nb + nc] = 1.0;
                Ab[nc * nb + r] = 1.0;
            }
            double* Bd = (double*)mem.alloc(nb * nb * sizeof(double));
            double* Bi = (double*)mem.alloc(nb * nb * sizeof(double));
            IIM_HIP(hipMemcpyAsync(Bd, Ab.data(), nb * nb * sizeof(double), hipMemcpyHostToDevice, stream));
            run_coarse_invert(Bd, Bi, nb, d_err, stream);
            IIM_HIP(hipMemcpy2DAsync(Ainv64, nc * sizeof(double), Bi, nb * sizeof(double), nc * sizeof(double), nc,
                                     hipMemcpyDeviceToDevice, stream));
            IIM_HIP(hipStreamSynchronize(stream));
            mem.release(Bi);
            mem.release(Bd);
        } else {
            run_coarse_invert(A, Ainv64, nc, d_err, stream);
        }
        run_convert<double, float>(Ainv64, Ainv32, nc * nc, 1.0, stream);
        mem.release(A);
        mem.release(d_col);
    }

    // ---- solve buffers: one zeroed block for the level-0 vectors and the
    // Krylov bases, one for the V-cycle vectors of every level
    const int64_t N = box.size();
    const int m = opt.restart;
    ldv = (krylov_len() + 63) / 64 * 64;
    {
        double* blk = (double*)mem.alloc((size_t)(2 * m + 6) * ldv * sizeof(double));
        IIM_HIP(hipMemsetAsync(blk, 0, (size_t)(2 * m + 6) * ldv * sizeof(double), stream));
        boxval = blk;
        rhs = blk + ldv;
        xk = blk + 2 * ldv;
        rk = blk + 3 * ldv;
        wk = blk + 4 * ldv;
        Vb = blk + 5 * ldv;
        Zb = Vb + (size_t)(m + 1) * ldv;
    }
    red_part = (double*)mem.alloc((size_t)(RED_PART_DOUBLES + 4 * 64 + 2) * sizeof(double));
    IIM_HIP(hipMemsetAsync(red_part, 0, (size_t)(RED_PART_DOUBLES + 4 * 64 + 2) * sizeof(double), stream));
    red_out = red_part + RED_PART_DOUBLES;
    red_scale = red_out + 4 * 64;
    const size_t tsz = opt.precision == IIM_PREC_FP64 ? sizeof(double) : sizeof(float);
    const size_t ssz = opt.precision == IIM_PREC_FP64 ? 8 : (opt.precision == IIM_PREC_MIXED32 ? 4 : 2);
    // levels small enough for the single-workgroup tail kernel
    // default: in 2D the fused LDS legs are faster than the one-workgroup tail on
    // every level but the coarsest; in 3D small levels go to the tail
    const int64_t tail_default = TAIL_MAX_NODES;
    const int64_t tail_max = opt.tail_nodes == 0 ? tail_default : (int64_t)opt.tail_nodes;
    tail_first = nl - 1;
    // the W-cycle visits every level from the host, and periodic levels take
    // the grid kernels (neighbours modulo n): the one-workgroup kernel then
    // holds the coarse solve only
    if (opt.cycle_gamma == 1 && !grid.periodic)
        while (tail_first > 0 && levels[tail_first - 1].box.size() <= tail_max) --tail_first;
    // 3D grid levels keep their vectors colour-split: a red-black half-sweep then
    // reads and writes whole contiguous colour rows
    for (int l = 0; l < nl; ++l) {
        Level& L = levels[l];
        L.hx = ((L.box.dims[0] + 1) / 2 + 3) / 4 * 4;
        L.half = (int64_t)L.hx * L.box.dims[1] * L.box.dims[2];
        L.split = dim == 3 && l < tail_first && opt_split && 2 * L.half <= (int64_t)INT32_MAX;
        if (L.split) {
            L.lab_split = (uint8_t*)mem.alloc(2 * L.half);
            run_box_to_level<uint8_t>(level_dev(l), L.labels, L.lab_split, stream);
        }
    }
    {
        const bool two = dim == 2 && opt_fused;
        auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
        size_t total = 0;
        for (Level& L : levels) total += up256(L.vsize() * ssz) * (two ? 2 : 1) + up256(L.vsize() * tsz);
        char* blk = (char*)mem.alloc(total);
        IIM_HIP(hipMemsetAsync(blk, 0, total, stream));  // entries of no node stay zero for good
        for (Level& L : levels) {
            L.z = blk;
            blk += up256(L.vsize() * ssz);
            L.b = blk;
            blk += up256(L.vsize() * tsz);
            if (two) {
                L.z2 = blk;
                blk += up256(L.vsize() * ssz);
            }
        }
    }
    // the tail runs in LDS when its levels' vectors fit
    {
        int64_t off = 0;
        auto up16 = [](int64_t v) { return (v + 15) / 16 * 16; };
        for (int l = tail_first; l < nl; ++l) off += up16(levels[l].box.size() * ssz) + up16(levels[l].box.size() * tsz);
        tail_lds_bytes = off <= TAIL_LDS_MAX ? off : 0;
        if (tail_lds_bytes) enable_tail_lds();
    }
    {
        TailDev T{};
        T.first = tail_first;
        T.last = nl - 1;
        T.mode = (side == IIM_SIDE_INTERFACE || bc == IIM_BC_DIRICHLET) ? 0 : 1;
        T.nu_pre = opt.nu_pre;
        T.nu_post = opt.nu_post;
        T.nc = nc;
        T.clist = coarse_list;
        T.Ainv = opt.precision == IIM_PREC_FP64 ? (const void*)Ainv64 : (const void*)Ainv32;
        int64_t off = 0;
        auto up16 = [](int64_t v) { return (v + 15) / 16 * 16; };
        for (int l = 0; l < nl; ++l) {
            T.lev[l] = level_dev(l);
            T.z[l] = levels[l].z;
            T.b[l] = levels[l].b;
            T.lds_z[l] = T.lds_b[l] = 0;
            if (l >= tail_first) {
                T.lds_z[l] = off;
                off += up16(levels[l].box.size() * ssz);
                T.lds_b[l] = off;
                off += up16(levels[l].box.size() * tsz);
            }
        }
        d_tail = (TailDev*)mem.alloc(sizeof(TailDev));
        IIM_HIP(hipMemcpyAsync(d_tail, &T, sizeof(TailDev), hipMemcpyHostToDevice, stream));
    }
    if (!hpin) hpin = take_hpin();
    for (int i = 0; i < 8; ++i) IIM_HIP(hipEventCreate(&ev[i]));
    for (int i = 0; i < 2; ++i) IIM_HIP(hipEventCreateWithFlags(&iter_done[i], hipEventDisableTiming));
    read_sc(1);  // [wait 6]
    raise_setup_error(err_bits(), "coarse inverse");
    mem.release(d_sc);
    t_setup_ms = now_ms() - t0;
}

LevelDev Problem::level_dev(int l) const {
    const Level& L = levels[l];
    LevelDev D;
    D.dim = dim;
    D.n = L.n;
    D.box = L.box;
    for (int d = 0; d < 3; ++d) {
        D.core_lo[d] = L.core_lo[d];
        D.core_hi[d] = L.core_hi[d];
    }
    D.labels = L.labels;
    D.irr_index = L.irr_index;
    D.rec64 = L.rec64;
    D.rec32 = L.rec32;
    D.split = L.split;
    D.hx = L.hx;
    D.half = L.half;
    D.lab_split = L.lab_split;
    D.periodic = grid.periodic ? 1 : 0;
    return D;
}

LevelSet Problem::level_set() const {
    LevelSet S{};
    for (size_t l = 0; l < levels.size() && l < (size_t)MAX_LEVELS; ++l) {
        S.g[l] = levels[l].geom;
        S.b[l] = levels[l].box;
        S.labels[l] = levels[l].labels;
        S.off[l] = 0;
    }
    return S;
}

GhostDev Problem::ghost_dev() const {
    GhostDev G;
    G.bc = bc;
    G.nsides = nsides;
    G.w = w;
    G.nrows = nrows_apply;
    G.beta_plus = opt.beta_plus;
    G.beta_minus = opt.beta_minus;
    G.ptr = ls_ptr;
    G.idx = ls_idx;
    G.W = W_apply;
    G.Sc = ls_Sc;
    G.dcoef = dcoef;
    G.nnz = nnz;
    G.ncp = cp.ncp;
    return G;
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------
void Problem::apply_box(const double* x, double* y, int with_data) {
    run_ghosts(ghost_dev(), x, cpdata, with_data, ghost, stream);
    const Level& L0 = levels[0];
    if (grid.periodic) {
        run_ho_apply_periodic(dim, box, grid.n, L0.labels, ho_irr_index, ho_slots, ho_nodes, ho_nirr, ghost,
                              1.0 / (h * h), opt.beta_plus, opt.beta_minus, x, y, stream);
        return;
    }
    run_ho_apply(dim, box, L0.core_lo, L0.core_hi, L0.labels, ho_irr_index, ho_slots, ho_nodes, ho_nirr, ghost, boxval,
                 w, 1.0 / (h * h),
                 opt.beta_plus, opt.beta_minus, x, y, with_data, stream);
}

void Problem::apply_op(double* x, double* y, const double* alpha_src) {
    apply_box(x, y, 0);
    if (singular) {
        const int64_t n = box.size();
        run_border(x, alpha_src ? alpha_src : x + n, levels[0].labels, n, y, red_part, stream);
    }
}

// fused pre-smoothing from a zero iterate + residual + restriction on level l
// (2D, one LDS-tiled kernel); false when it does not apply
template <typename T, typename S>
bool Problem::down_leg(int l, const CastInArgs* cast) {
    if (!opt_fused || dim != 2) return false;
    return run_down_fused<T, S>(level_dev(l), level_dev(l + 1), (const T*)levels[l].b, (S*)levels[l].z,
                                (T*)levels[l + 1].b, opt.nu_pre, stream, cast);
}

// fused prolongation + post-smoothing on level l (2D, one LDS-tiled kernel
// reading z and writing z2); returns the buffer holding the result, or nullptr
// when it does not apply
template <typename T, typename S>
const S* Problem::up_leg(int l, const S* zres, double* out) {
    if (!opt_fused || dim != 2 || !levels[l].z2) return nullptr;
    const int mode = (side == IIM_SIDE_INTERFACE || bc == IIM_BC_DIRICHLET) ? 0 : 1;
    S* z2 = (S*)levels[l].z2;
    return run_up_fused<T, S>(level_dev(l), level_dev(l + 1), mode, zres, (const T*)levels[l].b,
                              (const S*)levels[l].z, z2, opt.nu_post, stream, out, out ? red_scale + 1 : nullptr)
               ? z2
               : nullptr;
}

template <typename T, typename S>
void Problem::vcycle_t(const double* v, double* out, bool scaled, bool out_basis, int part) {
    const int nl = (int)levels.size();
    const int t = tail_first;
    LevelDev D0 = level_dev(0);
    if (part != 2) vcycle_down<T, S>(v, scaled);
    if (part == 0) {
        if (tail_runner)
            tail_runner->run(*this);
        else
            run_tail<T, S>(dim, d_tail, tail_lds_bytes, stream);  // levels t..nl-1, coarse solve included
    }
    if (part == 1) return;
    const int mode = (side == IIM_SIDE_INTERFACE || bc == IIM_BC_DIRICHLET) ? 0 : 1;
    const S* zres = (const S*)levels[t].z;  // result of the level below the current one
    bool have_out = false;
    for (int l = t - 1; l >= 0; --l) {
        // a basis column is zero off the core, so the last fused leg may write it directly
        double* o = (l == 0 && out_basis) ? out : nullptr;
        if (const S* r = up_leg<T, S>(l, zres, o)) {
            zres = r;
            have_out = o != nullptr;
            continue;
        }
        LevelDev D = level_dev(l), C = level_dev(l + 1);
        S* z = (S*)levels[l].z;
        T* b = (T*)levels[l].b;
        run_prolong<T, S>(D, C, mode, zres, z, stream);
        // the last half-sweep on a colour-split level 0 may write a basis column directly
        const bool fuse_out = l == 0 && out_basis && D.split && opt.nu_post > 0;
        for (int s = 0; s < opt.nu_post; ++s) {
            run_rbgs<T, S>(D, 0, z, b, stream);
            if (fuse_out && s == opt.nu_post - 1) {
                run_rbgs_out<T, S>(D, z, b, out, red_scale + 1, stream);
                have_out = true;
            } else {
                run_rbgs<T, S>(D, 1, z, b, stream);
            }
        }
        zres = z;
    }
    (void)nl;
    if (!have_out) run_cast_out<S>(D0, zres, red_scale + 1, out, stream);
}

// the levels above the tail of a V-cycle: input scaling and cast, then per
// level pre-smoothing from zero, residual and restriction
template <typename T, typename S>
void Problem::vcycle_down(const double* v, bool scaled) {
    const int t = tail_first;
    LevelDev D0 = level_dev(0);
    if (!scaled) run_absmax(v, box.size(), red_part, red_scale, stream);
    // the first fused leg makes level 0's right-hand side from v itself
    const CastInArgs cast{v, red_scale + 1, h * h, opt.beta_plus, opt.beta_minus};
    bool have_b = false;
    auto cast_in = [&]() {
        if (!have_b) run_cast_in<T>(D0, v, red_scale + 1, h * h, opt.beta_plus, opt.beta_minus, (T*)levels[0].b, stream);
        have_b = true;
    };
    // 3D colour-split levels start their pre-smoothing without a zero pass: the
    // first colour-0 half-sweep from zero (z = b / diag) is done by the pass that
    // makes b (the cast on level 0, the restriction below it)
    bool started = false;  // level l's iterate already holds its first half-sweep
    for (int l = 0; l < t; ++l) {
        if (down_leg<T, S>(l, l == 0 ? &cast : nullptr)) {
            have_b = true;
            continue;
        }
        LevelDev D = level_dev(l), C = level_dev(l + 1);
        S* z = (S*)levels[l].z;
        T* b = (T*)levels[l].b;
        const bool fuse = D.split && opt.nu_pre > 0;
        if (l == 0 && fuse && !have_b) {
            run_cast_sweep0<T, S>(D, v, red_scale + 1, h * h, opt.beta_plus, opt.beta_minus, b, z, stream);
            have_b = started = true;
        }
        cast_in();
        if (!started) run_zero<S>(z, levels[l].vsize(), stream);
        for (int s = 0; s < opt.nu_pre; ++s) {
            if (!(s == 0 && started)) run_rbgs<T, S>(D, 0, z, b, stream);
            run_rbgs<T, S>(D, 1, z, b, stream);
        }
        const bool next = dim == 3 && l + 1 < t && level_dev(l + 1).split && opt.nu_pre > 0;
        run_resid_restrict<T, S>(D, C, z, b, (T*)levels[l + 1].b, stream, next ? (S*)levels[l + 1].z : nullptr);
        started = next;
    }
    cast_in();  // every level in the tail
}

// One visit of level l in a W-cycle (cycle index 2): pre-smoothing from zero or
// from the iterate the previous visit left, residual + restriction, two visits
// of level l + 1 (the first from zero), prolongation + correction,
// post-smoothing.  The coarse solve ignores its start, so a second visit of the
// coarsest level would return the same iterate and is not made.  Every level
// runs its unfused kernels, which take any start.
template <typename T, typename S>
void Problem::wvisit(int l, bool zero_start) {
    const int nl = (int)levels.size();
    if (l == nl - 1) {
        run_tail<T, S>(dim, d_tail, tail_lds_bytes, stream);  // coarse solve only (tail_first = nl - 1)
        return;
    }
    LevelDev D = level_dev(l), C = level_dev(l + 1);
    S* z = (S*)levels[l].z;
    T* b = (T*)levels[l].b;
    if (zero_start) run_zero<S>(z, levels[l].vsize(), stream);
    for (int s = 0; s < opt.nu_pre; ++s) {
        run_rbgs<T, S>(D, 0, z, b, stream);
        run_rbgs<T, S>(D, 1, z, b, stream);
    }
    run_resid_restrict<T, S>(D, C, z, b, (T*)levels[l + 1].b, stream);
    wvisit<T, S>(l + 1, true);
    if (l + 1 < nl - 1) wvisit<T, S>(l + 1, false);
    const int mode = (side == IIM_SIDE_INTERFACE || bc == IIM_BC_DIRICHLET) ? 0 : 1;
    run_prolong<T, S>(D, C, mode, (const S*)levels[l + 1].z, z, stream);
    for (int s = 0; s < opt.nu_post; ++s) {
        run_rbgs<T, S>(D, 0, z, b, stream);
        run_rbgs<T, S>(D, 1, z, b, stream);
    }
}

template <typename T, typename S>
void Problem::wcycle_t(const double* v, double* out, bool scaled) {
    LevelDev D0 = level_dev(0);
    if (!scaled) run_absmax(v, box.size(), red_part, red_scale, stream);
    run_cast_in<T>(D0, v, red_scale + 1, h * h, opt.beta_plus, opt.beta_minus, (T*)levels[0].b, stream);
    wvisit<T, S>(0, true);
    run_cast_out<S>(D0, (const S*)levels[0].z, red_scale + 1, out, stream);
}

void Problem::vcycle(const double* v, double* out, bool scaled, bool out_basis, int part) {
    const bool w = opt.cycle_gamma == 2;
    if (w && part != 0) throw Error(IIM_E_INTERNAL, "the W-cycle runs whole");
    if (opt.precision == IIM_PREC_FP64) {
        if (w) wcycle_t<double, double>(v, out, scaled);
        else vcycle_t<double, double>(v, out, scaled, out_basis, part);
    } else if (opt.precision == IIM_PREC_MIXED32) {
        if (w) wcycle_t<float, float>(v, out, scaled);
        else vcycle_t<float, float>(v, out, scaled, out_basis, part);
    } else {
        if (w) wcycle_t<float, __half>(v, out, scaled);
        else vcycle_t<float, __half>(v, out, scaled, out_basis, part);
    }
}

// One inner FGMRES iteration on the device: z_j = M^{-1} v_j, w = A z_j,
// classical Gram-Schmidt against v_0..v_j, v_{j+1} = w / |w|, and the Hessenberg column copied to
// pinned host memory.  Pointers are fixed per j, so it can be captured.
void Problem::iteration_body(int j, hipEvent_t* evs, int part) {
    const int64_t N = krylov_len();
    double* vj = Vb + (size_t)j * ldv;
    double* zj = Zb + (size_t)j * ldv;
    vcycle(vj, zj, j > 0, true, part);  // v_j (j > 0) came from this cycle's fused pass, which left max |v_j|
    if (part == 1) return;
    if (evs) IIM_HIP(hipEventRecord(evs[1], stream));
    // bordered: the preconditioner is the identity on alpha, so z_j takes v_j's
    apply_op(zj, wk, vj + box.size());
    if (evs) IIM_HIP(hipEventRecord(evs[2], stream));
    // Classical Gram-Schmidt: h = V^T w (with |w|^2 when the second pass is
    // conditional); the second pass w -= V h with h' = V^T w and |w|^2 in the
    // same sweep, every iteration (CGS2) or only when the first pass left less
    // than 1e-2 of |w| (decided on the device, so launches stay queued); then
    // v_{j+1} = (w - V h') / |w - V h'|, the norm by Pythagoras.  The column's
    // record goes straight to pinned host memory (no copy).
    double* rec = hpin + (size_t)j * HCOL;
    const bool gated = opt.orthogonalisation == 1;
    run_multidot(Vb, ldv, j + 1, wk, N, red_part, red_out, stream, rec, gated ? 1 : 0);
    run_update_dot(Vb, ldv, j + 1, red_out, wk, N, j + 1, 1, red_part, red_out + 64, stream, rec + 64, gated);
    // the next cycle's input scale comes from the box entries only, as for v_0
    run_update_scale(Vb, ldv, j + 1, red_out + 64, wk, Vb + (size_t)(j + 1) * ldv, N, red_out + 128, red_part,
                     red_scale, stream, rec + 128, box.size());
}

// ---------------------------------------------------------------------------
// FGMRES(m), right preconditioned, classical Gram-Schmidt with a second pass
// every iteration or only where the first loses orthogonality; Givens
// rotations on the host.
// ---------------------------------------------------------------------------
int Problem::solve(double* u_full, const double* x0_full, double* hist, int hist_cap, iim_stats* st) {
    const double t0 = now_ms();
    const int64_t N = krylov_len();  // the box, plus alpha for a singular problem
    const int m = opt.restart;
    iim_stats S{};
    float t_apply = 0.f, t_vc = 0.f, t_kr = 0.f;
    if (x0_full) {
        run_full_to_box(dim, grid.n, box, x0_full, xk, levels[0].labels, 1, stream);
        if (singular) run_fill(xk + box.size(), 1, 0.0, stream);  // alpha starts at zero
    } else
        IIM_HIP(hipMemsetAsync(xk, 0, N * sizeof(double), stream));
    double bnorm2;
    run_norm2(rhs, N, red_part, red_out, stream);
    IIM_HIP(hipMemcpyAsync(&bnorm2, red_out, sizeof(double), hipMemcpyDeviceToHost, stream));
    IIM_HIP(hipStreamSynchronize(stream));
    const double bnorm = std::sqrt(bnorm2);
    int status = IIM_OK;
    int its = 0, cycles = 0, hl = 0, second_passes = 0;
    double true_rel = 0.0;
    std::vector<double> H((m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
    if (bnorm == 0.0) {
        IIM_HIP(hipMemsetAsync(xk, 0, N * sizeof(double), stream));
    } else {
        while (true) {
            // true residual r = b - A x
            apply_op(xk, wk);
            run_copy(rhs, rk, N, stream);
            run_axpby(-1.0, wk, 1.0, rk, N, stream);
            double rn2;
            run_norm2(rk, N, red_part, red_out, stream);
            IIM_HIP(hipMemcpyAsync(&rn2, red_out, sizeof(double), hipMemcpyDeviceToHost, stream));
            IIM_HIP(hipStreamSynchronize(stream));
            const double beta = std::sqrt(rn2);
            true_rel = beta / bnorm;
            if (!(true_rel == true_rel)) {
                status = IIM_E_BREAKDOWN;
                break;
            }
            if (true_rel <= opt.rtol) break;
            if (its >= opt.max_iters) {
                status = IIM_NOT_CONVERGED;
                break;
            }
            ++cycles;
            // v_0 = r / beta
            IIM_HIP(hipMemcpyAsync(red_out + 192, &rn2, sizeof(double), hipMemcpyHostToDevice, stream));
            run_normalize(rk, red_out + 192, Vb, N, stream);
            std::fill(gv.begin(), gv.end(), 0.0);
            gv[0] = beta;
            int k = 0;
            bool breakdown = false;
            // Iteration j+1 needs only device data of iteration j, so in graph mode
            // it is queued before the host reads column j: the host's wait and
            // its Givens update overlap the next iteration.  A queued iteration
            // past convergence writes only basis vectors the update never reads.
            // With a tail runner (serving) the iteration is captured as two
            // graphs, before and after the V-cycle's tail, and the runner runs
            // the tail between their launches.
            const bool split = tail_runner && opt.cycle_gamma == 1;
            auto capture = [&](hipGraphExec_t* slot, int jj, int part) {
                if (*slot) return;
                hipGraph_t g;
                IIM_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
                iteration_body(jj, nullptr, part);
                IIM_HIP(hipStreamEndCapture(stream, &g));
                IIM_HIP(hipGraphInstantiate(slot, g, nullptr, nullptr, 0));
                IIM_HIP(hipGraphDestroy(g));
            };
            const bool pipelined = opt.use_graph != 0;
            auto enqueue = [&](int jj) {
                if (opt.use_graph == 1 && split) {
                    capture(&pre_graph[jj], jj, 1);
                    capture(&iter_graph[jj], jj, 2);
                    IIM_HIP(hipGraphLaunch(pre_graph[jj], stream));
                    tail_runner->run(*this);
                    IIM_HIP(hipGraphLaunch(iter_graph[jj], stream));
                } else if (opt.use_graph == 1) {
                    capture(&iter_graph[jj], jj, 0);
                    IIM_HIP(hipGraphLaunch(iter_graph[jj], stream));
                } else {
                    iteration_body(jj);
                }
                IIM_HIP(hipEventRecord(iter_done[jj & 1], stream));
            };
            if (pipelined) {
                IIM_HIP(hipEventRecord(ev[0], stream));
                enqueue(0);
            }
            for (int j = 0; j < m; ++j) {
                if (pipelined) {
                    if (j + 1 < m && its + 1 < opt.max_iters) enqueue(j + 1);
                    IIM_HIP(hipEventSynchronize(iter_done[j & 1]));  // recorded after graph j, before j+1
                } else {
                    IIM_HIP(hipEventRecord(ev[0], stream));
                    iteration_body(j, ev);
                    IIM_HIP(hipEventRecord(ev[3], stream));
                    IIM_HIP(hipStreamSynchronize(stream));
                    float a1, a2, a3;
                    IIM_HIP(hipEventElapsedTime(&a1, ev[0], ev[1]));
                    IIM_HIP(hipEventElapsedTime(&a2, ev[1], ev[2]));
                    IIM_HIP(hipEventElapsedTime(&a3, ev[2], ev[3]));
                    t_vc += a1;
                    t_apply += a2;
                    t_kr += a3;
                }
                const double* hbuf = hpin + (size_t)j * HCOL;
                for (int i = 0; i <= j; ++i) H[i * m + j] = hbuf[i] + hbuf[64 + i];
                if (opt.orthogonalisation == 0 || hbuf[64 + 63] != 0.0) ++second_passes;
                const double hn = std::sqrt(hbuf[128]);
                H[(j + 1) * m + j] = hn;
                if (!(hn == hn)) {
                    breakdown = true;
                    break;
                }
                for (int i = 0; i < j; ++i) {
                    double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                    H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                    H[i * m + j] = t;
                }
                double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
                cs[j] = H[j * m + j] / den;
                sn[j] = H[(j + 1) * m + j] / den;
                H[j * m + j] = den;
                H[(j + 1) * m + j] = 0.0;
                gv[j + 1] = -sn[j] * gv[j];
                gv[j] = cs[j] * gv[j];
                ++its;
                k = j + 1;
                const double est = std::fabs(gv[j + 1]) / bnorm;
                if (hist && hl < hist_cap) hist[hl++] = est;
                if (est <= opt.rtol || its >= opt.max_iters || hn == 0.0) break;
            }
            if (pipelined) {
                // wait for the cycle's last queued iteration before the update
                IIM_HIP(hipEventRecord(ev[3], stream));
                IIM_HIP(hipEventSynchronize(ev[3]));
                float a;
                IIM_HIP(hipEventElapsedTime(&a, ev[0], ev[3]));
                t_kr += a;
            }
            if (breakdown) {
                status = IIM_E_BREAKDOWN;
                break;
            }
            for (int i = k - 1; i >= 0; --i) {
                double acc = gv[i];
                for (int l = i + 1; l < k; ++l) acc -= H[i * m + l] * y[l];
                y[i] = acc / H[i * m + i];
            }
            IIM_HIP(hipMemcpyAsync(red_out + 192, y.data(), k * sizeof(double), hipMemcpyHostToDevice, stream));
            run_axpy_multi(Zb, ldv, k, red_out + 192, xk, N, stream);
        }
    }
    if (u_full) run_box_to_full(dim, grid.n, box, xk, levels[0].labels, std::nan(""), u_full, stream);
    if (singular)
        IIM_HIP(hipMemcpyAsync(&S.shift_alpha, xk + box.size(), sizeof(double), hipMemcpyDeviceToHost, stream));
    IIM_HIP(hipStreamSynchronize(stream));
    S.bordered = singular ? 1 : 0;
    S.status = status;
    S.iterations = its;
    S.cycles = cycles;
    S.hist_len = hl;
    S.second_passes = second_passes;
    S.final_rel_residual = true_rel;
    S.t_solve_ms = now_ms() - t0;
    S.t_apply_ms = t_apply;
    S.t_vcycle_ms = t_vc;
    S.t_krylov_ms = t_kr;
    if (st) *st = S;
    return status;
}

// ---------------------------------------------------------------------------
// the caller's data (Sec. 2.1-2.3): boundary / interface values per control
// point and box-face values, then the right-hand side b = f - L_Gamma u_Gamma
// ---------------------------------------------------------------------------
void Problem::set_boundary_data(const double* cp_data, const double* box_data, int mem_kind, double* staging) {
    const int64_t ncd = cp.ncp * (bc == IIM_BC_JUMP ? 2 : 1);
    hipMemcpyKind k = mem_kind == IIM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (ncd) {
        if (!cp_data) throw Error(IIM_E_INVALID_ARG, "cp_data is required");
        IIM_HIP(hipMemcpyAsync(cpdata, cp_data, ncd * sizeof(double), k, stream));
    }
    if (box_data) {
        const int64_t n1 = grid.n + 1;
        const int64_t tot = dim == 2 ? n1 * n1 : n1 * n1 * n1;
        double* tmp = staging ? staging : (double*)mem.alloc(tot * sizeof(double));
        IIM_HIP(hipMemcpyAsync(tmp, box_data, tot * sizeof(double), k, stream));
        run_full_to_box(dim, grid.n, box, tmp, boxval, levels[0].labels, 2, stream);
        IIM_HIP(hipStreamSynchronize(stream));
        if (!staging) mem.release(tmp);
    } else {
        IIM_HIP(hipMemsetAsync(boxval, 0, box.size() * sizeof(double), stream));
    }
    IIM_HIP(hipStreamSynchronize(stream));
}

void Problem::set_rhs(const double* f, int mem_kind) {
    if (!f) throw Error(IIM_E_INVALID_ARG, "null argument");
    const int64_t n1 = grid.n + 1;
    const int64_t tot = dim == 2 ? n1 * n1 : n1 * n1 * n1;
    const double* src = f;
    double* tmp = nullptr;
    if (mem_kind != IIM_MEM_DEVICE) {
        tmp = (double*)mem.alloc(tot * sizeof(double));
        IIM_HIP(hipMemcpyAsync(tmp, f, tot * sizeof(double), hipMemcpyHostToDevice, stream));
        src = tmp;
    }
    // b = f - L_Gamma u_Gamma = f - apply(0, with data)
    run_full_to_box(dim, grid.n, box, src, rhs, levels[0].labels, 1, stream);
    IIM_HIP(hipMemsetAsync(xk, 0, box.size() * sizeof(double), stream));
    apply_box(xk, wk, 1);
    run_axpby(-1.0, wk, 1.0, rhs, box.size(), stream);
    IIM_HIP(hipStreamSynchronize(stream));
    if (tmp) mem.release(tmp);
}

// ---------------------------------------------------------------------------
// manufactured data and its error (benchmarks and serving)
// ---------------------------------------------------------------------------
void Problem::synth_data(int kind) {
    if (kind != 1) throw Error(IIM_E_INVALID_ARG, "unknown synthetic data kind");
    const int64_t N = box.size();
    run_synth_cp(kind, dim, bc, cp, opt.beta_plus, opt.beta_minus, cpdata, stream);
    run_synth_nodes(kind, levels[0].geom, box, levels[0].labels, opt.beta_plus, opt.beta_minus, rhs, boxval, stream);
    // b = f - L_Gamma u_Gamma, as for caller-supplied data
    IIM_HIP(hipMemsetAsync(xk, 0, N * sizeof(double), stream));
    apply_box(xk, wk, 1);
    run_axpby(-1.0, wk, 1.0, rhs, N, stream);
}

double Problem::synth_error(int kind, const double* u_full) {
    if (kind != 1) throw Error(IIM_E_INVALID_ARG, "unknown synthetic data kind");
    unsigned long long* d = (unsigned long long*)(red_out + 250);
    // a singular problem's u is fixed only up to a constant: its error is
    // measured after removing the mean of u - u_exact over the unknowns
    double shift = 0.0;
    if (singular) {
        const int nb = run_synth_diff_sum(kind, levels[0].geom, box, levels[0].labels, u_full, red_part, stream);
        std::vector<double> part(2 * (size_t)nb);
        IIM_HIP(hipMemcpyAsync(part.data(), red_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
        IIM_HIP(hipStreamSynchronize(stream));
        double sum = 0.0, cnt = 0.0;
        for (int i = 0; i < nb; ++i) {
            sum += part[2 * i];
            cnt += part[2 * i + 1];
        }
        if (cnt > 0.0) shift = sum / cnt;
    }
    IIM_HIP(hipMemsetAsync(d, 0, sizeof(unsigned long long), stream));
    run_synth_err(kind, levels[0].geom, box, levels[0].labels, u_full, d, stream, shift);
    unsigned long long bits = 0;
    IIM_HIP(hipMemcpyAsync(&bits, d, sizeof(bits), hipMemcpyDeviceToHost, stream));
    IIM_HIP(hipStreamSynchronize(stream));
    if (bits == ~0ull) return std::nan("");
    double v;
    std::memcpy(&v, &bits, sizeof(v));
    return v;
}

// ---------------------------------------------------------------------------
// Device bytes of a problem at its peak, before any device work: the storage
// boxes from a bounding box of the body (interior problems) or the whole grid,
// control points from the number of grid lines that cross the bounding
// spheres, least-squares entries from the largest set size of the default
// half-ellipse.  Upper estimates; every term is listed in the same order as the
// allocations of setup().
// ---------------------------------------------------------------------------
int64_t estimate_bytes(const iim_grid& g, const iim_geometry& geo, const iim_options& o) {
    const int dim = g.dim;
    const double h = (g.hi - g.lo) / g.n;
    const double PI = 3.14159265358979323846;
    // bounding spheres of the body
    std::vector<std::pair<std::vector<double>, double>> balls;
    if (geo.kind == IIM_GEOM_SPHERE) {
        balls.push_back({std::vector<double>(geo.params, geo.params + dim), geo.params[dim]});
    } else if (geo.kind == IIM_GEOM_STAR2D) {
        balls.push_back({{geo.params[0], geo.params[1]}, geo.params[2] + std::fabs(geo.params[3])});
    } else {
        int cnt = (int)std::llround(geo.params[0]);
        for (int s = 0; s < cnt; ++s) {
            const double* q = geo.params + 1 + (dim + 1) * s;
            balls.push_back({std::vector<double>(q, q + dim), q[dim]});
        }
    }
    // level-0 storage box
    int64_t dims[3] = {1, 1, 1};
    for (int d = 0; d < dim; ++d) {
        int64_t lo = 0, hi = g.n;
        if (geo.side == IIM_SIDE_INTERIOR && !balls.empty()) {
            double a = 1e300, b = -1e300;
            for (auto& bl : balls) {
                a = std::min(a, bl.first[d] - bl.second);
                b = std::max(b, bl.first[d] + bl.second);
            }
            lo = std::max<int64_t>(0, (int64_t)std::floor((a - g.lo) / h));
            hi = std::min<int64_t>(g.n, (int64_t)std::ceil((b - g.lo) / h));
        }
        dims[d] = hi - lo + 1 + 2 * (o.order_n / 2);  // level-0 padding: the stencil's reach
    }
    const int m = o.restart;
    const int64_t tsz = o.precision == IIM_PREC_FP64 ? 8 : 4;
    const int64_t ssz = o.precision == IIM_PREC_FP64 ? 8 : (o.precision == IIM_PREC_MIXED32 ? 4 : 2);
    const int64_t N0 = dims[0] * dims[1] * dims[2];
    // per node of level 0: labels, HO and SW irregular indices, 5 work vectors,
    // the Krylov bases V (m+1) and Z (m), the V-cycle iterate and right-hand side
    const int64_t zbufs = (dim == 2 && o.fused_smoothing) ? 2 : 1;  // second iterate buffer of the fused 2D legs
    // entries of a level vector: colour-split 3D levels round each box row up to even
    auto vec = [&](const int64_t* d) {
        return dim == 3 ? 2 * (((d[0] + 1) / 2 + 3) / 4 * 4) * d[1] * d[2] : d[0] * d[1] * d[2];
    };
    // (3D: the colour-split labels, one byte per vector entry)
    const int64_t lsplit = dim == 3 ? 1 : 0;
    int64_t bytes = N0 * (1 + 4 + 4 + 5 * 8 + (2 * m + 1) * 8) + vec(dims) * (zbufs * ssz + tsz + lsplit) +
                    (2 * m + 1) * 64 * 8;
    // setup transients alive together: the crossing flags and one selection
    // output per axis, the selections' scratch
    bytes += N0 * 5 * dim + SEL_BLOCKS * SEL_MAX * 4;
    // coarse levels: labels, SW index, iterate, right-hand side
    int64_t cd[3] = {dims[0], dims[1], dims[2]};
    int n = g.n;
    int64_t last = N0;
    while (n > o.coarsest_n) {
        n = (n + 1) / 2;
        for (int d = 0; d < dim; ++d) cd[d] = (cd[d] - 4) / 2 + 1 + 2 + 2;
        last = cd[0] * cd[1] * cd[2];
        bytes += last * (1 + 4) + vec(cd) * (zbufs * ssz + tsz + lsplit);
    }
    // coarsest dense inverse (A, FP64 and FP32 inverses, column map)
    const int64_t nc = std::min<int64_t>(last, 4096);
    bytes += nc * nc * (8 + 8 + 4) + last * 4;
    // control points: per line crossing of each bounding sphere
    double ncp = 0.0;
    for (auto& bl : balls) {
        const double r = bl.second / h + 1.0;
        ncp += dim == 2 ? 2.0 * 2.0 * (2.0 * r + 1.0) : 3.0 * 2.0 * PI * r * r;
    }
    if (geo.kind == IIM_GEOM_STAR2D) ncp *= 2.0;  // lobes lengthen the curve
    ncp = 1.15 * ncp + 64.0;
    const int ns = geo.side == IIM_SIDE_INTERFACE ? 2 : 1;
    const int w = o.order_n / 2;
    const int nrows = w + (geo.bc == IIM_BC_DIRICHLET ? 0 : 1);
    const double mset = dim == 2 ? (o.order_k == 7 ? 112.0 : 56.0) : (o.order_k == 7 ? 700.0 : 264.0);
    const double ncs = ncp * ns;
    bytes += (int64_t)(ncp * (4 + 4 + 24 + 24 + 8 + 16) + ncs * (4 + 4 + 8 * w * 2 + 8 * nrows + 4 + 4 + 1 + 8));
    bytes += (int64_t)(ncs * mset * (4 + 8 * nrows + (geo.bc == IIM_BC_NEUMANN ? 8 * w : 0)));
    // staging of the fits: a fixed segment of 64 * (rows per lane) entries per fit
    bytes += (int64_t)(ncs * (dim == 2 ? 128 : 256) * (4 + 8 * nrows));
    // scratch of oversized least-squares sets (one slab per wave, LS_SCRATCH_WAVES at most)
    const int K = o.order_k;
    const int p = dim == 2 ? K * (K + 1) / 2 : K * (K + 1) * (K + 2) / 6;
    bytes += (int64_t)std::min((double)LS_SCRATCH_WAVES, ncs) * (p + 4) * (dim == 2 ? 192 : 768) * 8;
    // irregular records: high-order slots (at most w nodes per crossing and side),
    // Shortley-Weller rows in FP64 and FP32 (at most one node per crossing, all levels)
    bytes += (int64_t)(ncs * (w * (2 * dim + 1) * 4 + 2 * (1 + 2 * dim) * 12));
    // reductions and small tables
    bytes += RED_PART_DOUBLES * 8 + 4096;
    return bytes + (4 << 20);
}

// ---------------------------------------------------------------------------
// level operations for tests (FP64 in and out, the handle's precision inside)
// ---------------------------------------------------------------------------
template <typename T, typename S>
int Problem::level_op_t(int l, int op, const double* in1, double* out) {
    const int nl = (int)levels.size();
    if (l < 0 || l >= nl) throw Error(IIM_E_INVALID_ARG, "level out of range");
    if (op == 2 && l == nl - 1) throw Error(IIM_E_INVALID_ARG, "no coarser level");
    if (op == 3 && l == 0) throw Error(IIM_E_INVALID_ARG, "no finer level");
    if (op == 4 && l != nl - 1) throw Error(IIM_E_INVALID_ARG, "coarse solve only on the coarsest level");
    if (op < 0 || op > 4) throw Error(IIM_E_INVALID_ARG, "bad op");
    std::vector<void*> tmp;
    auto alloc = [&](int64_t n, size_t sz) {
        void* p = mem.alloc((size_t)std::max<int64_t>(n, 1) * sz);
        IIM_HIP(hipMemsetAsync(p, 0, (size_t)std::max<int64_t>(n, 1) * sz, stream));
        tmp.push_back(p);
        return p;
    };
    // grid function (full grid, FP64) -> level vector of type U (level layout, scaled)
    auto to_level = [&](int lv, const double* full, double scale, auto* dst) {
        using U = std::remove_pointer_t<decltype(dst)>;
        const Level& L = levels[lv];
        const LevelDev D = level_dev(lv);
        double* box64 = (double*)alloc(L.box.size(), sizeof(double));
        double* lev64 = (double*)alloc(L.vsize(), sizeof(double));
        run_full_to_box(dim, L.n, L.box, full, box64, L.labels, 1, stream);
        run_box_to_level<double>(D, box64, lev64, stream);
        run_convert<double, U>(lev64, dst, L.vsize(), scale, stream);
    };
    // level vector of type U -> grid function (zero off the level's unknowns)
    auto from_level = [&](int lv, const auto* src, double scale, double* full) {
        using U = std::remove_const_t<std::remove_pointer_t<decltype(src)>>;
        const Level& L = levels[lv];
        const LevelDev D = level_dev(lv);
        double* lev64 = (double*)alloc(L.vsize(), sizeof(double));
        double* box64 = (double*)alloc(L.box.size(), sizeof(double));
        run_convert<U, double>(src, lev64, L.vsize(), scale, stream);
        run_level_to_box<double>(D, lev64, box64, stream);
        run_box_to_full(dim, L.n, L.box, box64, L.labels, 0.0, full, stream);
    };
    Level& L = levels[l];
    const int64_t vs = L.vsize();
    const double h2 = L.h * L.h;
    T* tb = (T*)alloc(vs, sizeof(T));
    S* tz = (S*)alloc(vs, sizeof(S));
    const LevelDev D = level_dev(l);
    const int mode = (side == IIM_SIDE_INTERFACE || bc == IIM_BC_DIRICHLET) ? 0 : 1;
    if (op == 0) {  // out = A_l in1
        to_level(l, in1, 1.0, tz);
        run_sw_apply<T, S>(D, tz, tb, stream);
        from_level(l, (const T*)tb, 1.0 / h2, out);
    } else if (op == 1) {  // one red-black sweep on out with right-hand side in1
        to_level(l, in1, h2, tb);
        to_level(l, out, 1.0, tz);
        run_rbgs<T, S>(D, 0, tz, tb, stream);
        run_rbgs<T, S>(D, 1, tz, tb, stream);
        from_level(l, (const S*)tz, 1.0, out);
    } else if (op == 2) {  // out(l+1) = half-weighting of in1
        to_level(l, in1, 1.0, tb);
        T* cb = (T*)alloc(levels[l + 1].vsize(), sizeof(T));
        run_resid_restrict<T, S>(D, level_dev(l + 1), tz, tb, cb, stream);
        from_level(l + 1, (const T*)cb, 0.25, out);
    } else if (op == 3) {  // out(l-1) = prolongation of in1
        to_level(l, in1, 1.0, tz);
        S* fz = (S*)alloc(levels[l - 1].vsize(), sizeof(S));
        run_prolong<T, S>(level_dev(l - 1), D, mode, tz, fz, stream);
        from_level(l - 1, (const S*)fz, 1.0, out);
    } else {  // coarse direct solve
        to_level(l, in1, h2, tb);
        const T* Ainv = std::is_same<T, double>::value ? (const T*)Ainv64 : (const T*)Ainv32;
        run_coarse_solve<T, S>(D, coarse_list, nc, Ainv, tb, tz, stream);
        from_level(l, (const S*)tz, 1.0, out);
    }
    IIM_HIP(hipStreamSynchronize(stream));
    for (void* p : tmp) mem.release(p);
    return IIM_OK;
}

template <typename T, typename S>
void Problem::launch_kernel_t(int kernel) {
    const int64_t N = box.size();
    switch (kernel) {
        case 0:
        case 11: {
            const Level& L0 = levels[0];
            if (grid.periodic) {
                if (kernel == 11 && dim == 2)
                    throw Error(IIM_E_INVALID_ARG, "2D periodic problems have no irregular-node kernel");
                run_ho_apply_periodic(dim, box, grid.n, L0.labels, ho_irr_index, ho_slots, ho_nodes, ho_nirr, ghost,
                                      1.0 / (h * h), opt.beta_plus, opt.beta_minus, rk, wk, stream,
                                      kernel == 0 ? 1 : 2);
                break;
            }
            run_ho_apply(dim, box, L0.core_lo, L0.core_hi, L0.labels, ho_irr_index, ho_slots, ho_nodes, ho_nirr, ghost,
                         boxval, w, 1.0 / (h * h), opt.beta_plus, opt.beta_minus, rk, wk, 0, stream,
                         kernel == 0 ? 1 : 2);
            break;
        }
        case 1: run_ghosts(ghost_dev(), rk, cpdata, 0, ghost, stream); break;
        case 2:
            run_rbgs<T, S>(level_dev(0), 0, (S*)levels[0].z, (const T*)levels[0].b, stream);
            run_rbgs<T, S>(level_dev(0), 1, (S*)levels[0].z, (const T*)levels[0].b, stream);
            break;
        case 3:
            if (levels.size() > 1)
                run_resid_restrict<T, S>(level_dev(0), level_dev(1), (const S*)levels[0].z, (const T*)levels[0].b,
                                         (T*)levels[1].b, stream);
            break;
        case 4:
            if (levels.size() > 1)
                run_prolong<T, S>(level_dev(0), level_dev(1), (side == IIM_SIDE_INTERFACE || bc == IIM_BC_DIRICHLET) ? 0 : 1,
                                  (const S*)levels[1].z, (S*)levels[0].z, stream);
            break;
        case 5: {
            int k = std::min(6, opt.restart);
            run_update_dot_stage1(Vb, ldv, k, red_out + 192, wk, N, k, 0, red_part, stream);
            break;
        }
        case 6: vcycle(rk, wk); break;
        case 7: apply_box(rk, wk, 0); break;
        case 8:
        case 9: {
            // the fused legs of level 0 (1 -> 0 reads level 1's iterate as the coarse result)
            if (levels.size() < 2 || tail_first < 1) throw Error(IIM_E_INVALID_ARG, "no fused leg on this problem");
            bool ok = kernel == 8 ? down_leg<T, S>(0, nullptr) : up_leg<T, S>(0, (const S*)levels[1].z, nullptr) != nullptr;
            if (!ok) throw Error(IIM_E_INVALID_ARG, "no fused leg on this problem");
            break;
        }
        default: throw Error(IIM_E_INVALID_ARG, "unknown kernel id");
    }
}

double Problem::time_kernel(int kernel, int reps) {
    // operands: deterministic non-trivial contents; red_out[192..] holds zeros (update coefficients)
    IIM_HIP(hipMemsetAsync(red_out + 192, 0, 32 * sizeof(double), stream));
    run_copy(rhs, rk, box.size(), stream);
    auto launch = [&]() {
        if (opt.precision == IIM_PREC_FP64) launch_kernel_t<double, double>(kernel);
        else if (opt.precision == IIM_PREC_MIXED32) launch_kernel_t<float, float>(kernel);
        else launch_kernel_t<float, __half>(kernel);
    };
    launch();  // warm
    IIM_HIP(hipEventRecord(ev[4], stream));
    for (int r = 0; r < reps; ++r) launch();
    IIM_HIP(hipEventRecord(ev[5], stream));
    IIM_HIP(hipEventSynchronize(ev[5]));
    float ms = 0.f;
    IIM_HIP(hipEventElapsedTime(&ms, ev[4], ev[5]));
    return (double)ms / reps;
}

int Problem::level_op(int l, int op, const double* in1, double* out) {
    if (opt.precision == IIM_PREC_FP64) return level_op_t<double, double>(l, op, in1, out);
    if (opt.precision == IIM_PREC_MIXED32) return level_op_t<float, float>(l, op, in1, out);
    return level_op_t<float, __half>(l, op, in1, out);
}

// A singular problem (interior domain, Neumann boundary) is bordered with one
// constant (Sec. 2.3), which fixes the null space of a connected domain only.
// The interior of a sphere union is connected exactly when the overlap graph of
// its spheres is (two balls overlap when their centres are closer than the sum
// of their radii); anything else is rejected here.
void check_singular_connected(const iim_grid& g, const iim_geometry& geo) {
    if (geo.kind != IIM_GEOM_SPHERE_UNION || geo.side != IIM_SIDE_INTERIOR || geo.bc != IIM_BC_NEUMANN) return;
    const int cnt = (int)geo.params[0], d = g.dim;
    std::vector<int> parent(std::max(cnt, 0));
    for (int i = 0; i < cnt; ++i) parent[i] = i;
    auto find = [&](int i) {
        while (parent[i] != i) i = parent[i] = parent[parent[i]];
        return i;
    };
    int comps = cnt;
    for (int i = 0; i < cnt; ++i)
        for (int j = i + 1; j < cnt; ++j) {
            const double* a = geo.params + 1 + i * (d + 1);
            const double* b = geo.params + 1 + j * (d + 1);
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) d2 += (a[k] - b[k]) * (a[k] - b[k]);
            const double rr = a[d] + b[d];
            if (d2 < rr * rr) {
                const int ri = find(i), rj = find(j);
                if (ri != rj) {
                    parent[ri] = rj;
                    --comps;
                }
            }
        }
    if (comps > 1)
        throw Error(IIM_E_INVALID_ARG,
                    "interior Neumann sphere union is not connected: the bordered system fixes one constant, "
                    "but each of the " + std::to_string(comps) + " components has its own");
}

std::unique_ptr<Problem> make_problem(const iim_grid* g, const iim_geometry* geo, const iim_options* opt,
                                      hipStream_t stream, double* hpin) {
    if (!g || !geo) throw Error(IIM_E_INVALID_ARG, "null argument");
    iim_options o;
    if (opt) o = *opt; else iim_default_options(&o);
    if (g->dim != 2 && g->dim != 3) throw Error(IIM_E_INVALID_ARG, "dim must be 2 or 3");
    if (g->n < 8 || g->n > 16384) throw Error(IIM_E_INVALID_ARG, "n out of range");
    if (!(g->hi > g->lo)) throw Error(IIM_E_INVALID_ARG, "empty domain");
    const bool o45 = o.order_n == 4 && o.order_k == 5, o67 = o.order_n == 6 && o.order_k == 7;
    if (!o45 && !o67) throw Error(IIM_E_INVALID_ARG, "built discretisations: (4,5) and (6,7)");
    if (o.restart < 1 || o.restart > 11) throw Error(IIM_E_INVALID_ARG, "restart must be in [1, 11]");
    if (o.use_graph < 0 || o.use_graph > 2) throw Error(IIM_E_INVALID_ARG, "use_graph must be 0, 1 or 2");
    if (o.orthogonalisation < 0 || o.orthogonalisation > 1)
        throw Error(IIM_E_INVALID_ARG, "orthogonalisation must be 0 or 1");
    if (o.cycle_gamma < 1 || o.cycle_gamma > 2) throw Error(IIM_E_INVALID_ARG, "cycle_gamma must be 1 (V) or 2 (W)");
    if (o.coarsest_n < 2) throw Error(IIM_E_INVALID_ARG, "coarsest_n must be >= 2");
    if (o.precision < 0 || o.precision > 2) throw Error(IIM_E_INVALID_ARG, "bad precision");
    if (!(o.beta_plus > 0) || !(o.beta_minus > 0)) throw Error(IIM_E_INVALID_ARG, "beta must be positive");
    if ((geo->side == IIM_SIDE_INTERFACE) != (geo->bc == IIM_BC_JUMP))
        throw Error(IIM_E_INVALID_ARG, "jump conditions go with interface problems");
    if (geo->kind < 0 || geo->kind > 3 || geo->side < 0 || geo->side > 2 || geo->bc < 0 || geo->bc > 2)
        throw Error(IIM_E_INVALID_ARG, "bad geometry enums");
    if (!geo->params) throw Error(IIM_E_INVALID_ARG, "null params");
    if (geo->kind == IIM_GEOM_STAR2D && (g->dim != 2 || geo->nparams < 5))
        throw Error(IIM_E_INVALID_ARG, "star needs dim 2 and 5 parameters");
    if (geo->kind == IIM_GEOM_SPHERE && geo->nparams < g->dim + 1)
        throw Error(IIM_E_INVALID_ARG, "sphere needs dim + 1 parameters");
    if (geo->kind == IIM_GEOM_SPHERE_UNION &&
        (geo->nparams < 1 || geo->params[0] < 0 || geo->nparams < 1 + (g->dim + 1) * (int)geo->params[0]))
        throw Error(IIM_E_INVALID_ARG, "sphere union parameter count");
    check_singular_connected(*g, *geo);
    if (g->periodic) {
        if (!o45) throw Error(IIM_E_INVALID_ARG, "periodic problems: the (4,5) scheme");
        if (g->n < 32) throw Error(IIM_E_INVALID_ARG, "periodic problems need n >= 32");
    }
    if (geo->kind == IIM_GEOM_GYROID && (g->dim != 3 || geo->nparams < 4 || !g->periodic))
        throw Error(IIM_E_INVALID_ARG, "the gyroid needs dim 3, 4 parameters and a periodic grid");
    if (geo->side != IIM_SIDE_INTERIOR || g->periodic) {
        // box faces (periodic images) must coincide on every level
        int n = g->n;
        while (n > o.coarsest_n) {
            if (n % 2) throw Error(IIM_E_INVALID_ARG, "exterior/interface problems need n = m 2^L with m <= coarsest_n");
            n /= 2;
        }
    }
    int dev = 0;
    IIM_HIP(hipGetDevice(&dev));
    configure_pool(dev);
    auto p = std::make_unique<Problem>();
    p->stream = stream;
    if (!p->stream) {
        // a blocking stream of our own: ordered with the legacy default stream,
        // and capturable (the default stream is not)
        p->stream = take_stream(dev);
        p->own_stream = true;
    }
    p->mem.stream = p->stream;
    p->mem.device = dev;
    if (hpin) {
        p->hpin = hpin;
        p->own_hpin = false;
    }
    p->grid = *g;
    p->opt = o;
    p->dim = g->dim;
    p->kind = geo->kind;
    p->side = geo->side;
    p->bc = geo->bc;
    // no Dirichlet value pins the constant: an interior Neumann domain, or a
    // periodic one whose immersed condition is Neumann or a jump
    p->singular = g->periodic ? geo->bc != IIM_BC_DIRICHLET
                              : (geo->side == IIM_SIDE_INTERIOR && geo->bc == IIM_BC_NEUMANN);
    p->params.assign(geo->params, geo->params + geo->nparams);
    // the fused legs start from zero; periodic levels keep the box layout and the
    // per-node grid kernels
    p->opt_fused = o.fused_smoothing != 0 && o.cycle_gamma == 1 && !g->periodic;
    p->opt_split = o.colour_split != 0;
    p->setup();
    return p;
}

Problem::~Problem() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& g : iter_graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& g : pre_graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (int i = 0; i < 8; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    for (int i = 0; i < 2; ++i)
        if (iter_done[i]) (void)hipEventDestroy(iter_done[i]);
    if (hpin && own_hpin) give_hpin(hpin);
    mem.release_all();
    if (stream) (void)hipStreamSynchronize(stream);
    if (own_stream && stream) give_stream(mem.device, stream);
}

}  // namespace iim

// ===========================================================================
// C ABI
// ===========================================================================
using namespace iim;

// Staging array of iim_set_boundary_data_noalloc: one copy per device, held
// until the process ends.  Host code never uses the name `scratch` as an
// address; it uses the per-device pointer from hipGetSymbolAddress, taken once
// per device (with that device current) on the first call there.
static __device__ __align__(256) double scratch[IIM_NOALLOC_MAX_NODES];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[64] = {};

static double* noalloc_scratch(int dev) {
    if (dev < 0 || dev >= 64) throw Error(IIM_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        IIM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error(IIM_E_DEVICE, "no address for the static staging array");
        g_scratch_ptr[dev] = (double*)ptr;
    }
    return g_scratch_ptr[dev];
}

struct iim_problem {
    std::unique_ptr<Problem> p;
};

#define ABI_TRY(...)                                               \
    try {                                                          \
        __VA_ARGS__;                                               \
    } catch (const iim::Error& e) {                                \
        iim::set_error(e.what());                                  \
        return e.code;                                             \
    } catch (const std::exception& e) {                            \
        iim::set_error(std::string("internal error: ") + e.what()); \
        return IIM_E_INTERNAL;                                     \
    } catch (...) {                                                \
        iim::set_error("internal error");                          \
        return IIM_E_INTERNAL;                                     \
    }

extern "C" {

int iim_default_options(iim_options* o) {
    if (!o) return IIM_E_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->order_n = 4;
    o->order_k = 5;
    o->beta_plus = 1.0;
    o->beta_minus = 1.0;
    o->rtol = 1e-10;
    o->max_iters = 500;
    o->restart = 10;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->coarsest_n = 8;
    o->precision = IIM_PREC_FP64;
    o->ls_axis_t = 0.0;
    o->ls_axis_n = 0.0;
    o->use_graph = 2;
    o->tail_nodes = 0;
    o->fused_smoothing = 1;
    o->colour_split = 1;
    o->orthogonalisation = 1;
    o->cycle_gamma = 1;
    return IIM_OK;
}

const char* iim_last_error(void) { return iim::last_error(); }

int iim_create(const iim_grid* g, const iim_geometry* geo, const iim_options* opt, void* stream, iim_problem** out) {
    ABI_TRY({
        iim::set_error("");
        if (!out) throw Error(IIM_E_INVALID_ARG, "null argument");
        *out = nullptr;
        auto p = make_problem(g, geo, opt, (hipStream_t)stream, nullptr);
        auto* h = new iim_problem;
        h->p = std::move(p);
        *out = h;
        return IIM_OK;
    })
}

void iim_destroy(iim_problem* p) {
    if (!p) return;
    try {
        if (p->p) (void)hipStreamSynchronize(p->p->stream);
    } catch (...) {
    }
    delete p;
}

int iim_get_info(const iim_problem* h, iim_info* info) {
    ABI_TRY({
        if (!h || !info) throw Error(IIM_E_INVALID_ARG, "null argument");
        const Problem& p = *h->p;
        std::memset(info, 0, sizeof(*info));
        info->dim = p.dim;
        info->n = p.grid.n;
        info->levels = (int)p.levels.size();
        info->sides = p.nsides;
        info->n_unknowns = p.levels[0].nunk;
        info->n_control_points = p.cp.ncp;
        info->n_ls_entries = p.nnz;
        info->n_irregular = p.ho_nirr;
        for (int d = 0; d < 3; ++d) {
            info->box_lo[d] = p.box.lo[d];
            info->box_dims[d] = p.box.dims[d];
        }
        info->device_bytes = (int64_t)p.mem.peak;
        info->t_setup_ms = p.t_setup_ms;
        return IIM_OK;
    })
}

int iim_control_points(const iim_problem* h, int64_t* count, double* xyz, double* normal) {
    ABI_TRY({
        if (!h || !count) throw Error(IIM_E_INVALID_ARG, "null argument");
        const Problem& p = *h->p;
        *count = p.cp.ncp;
        if (!xyz && !normal) return IIM_OK;
        const int64_t n = p.cp.ncp;
        std::vector<double> x(3 * n), nv(3 * n);
        IIM_HIP(hipMemcpyAsync(x.data(), p.cp.x, 3 * n * sizeof(double), hipMemcpyDeviceToHost, p.stream));
        IIM_HIP(hipMemcpyAsync(nv.data(), p.cp.n, 3 * n * sizeof(double), hipMemcpyDeviceToHost, p.stream));
        IIM_HIP(hipStreamSynchronize(p.stream));
        for (int64_t c = 0; c < n; ++c)
            for (int d = 0; d < p.dim; ++d) {
                if (xyz) xyz[c * p.dim + d] = x[d * n + c];
                if (normal) normal[c * p.dim + d] = nv[d * n + c];
            }
        return IIM_OK;
    })
}

static void labels_to_full(const Problem& p, int level, uint8_t* out) {
    const Level& L = p.levels[level];
    std::vector<uint8_t> lab(L.box.size());
    IIM_HIP(hipMemcpyAsync(lab.data(), L.labels, lab.size(), hipMemcpyDeviceToHost, p.stream));
    IIM_HIP(hipStreamSynchronize(p.stream));
    const int64_t n1 = L.n + 1;
    const int64_t tot = p.dim == 2 ? n1 * n1 : n1 * n1 * n1;
    for (int64_t f = 0; f < tot; ++f) {
        int ijk[3] = {(int)(f % n1), (int)((f / n1) % n1), p.dim == 3 ? (int)(f / (n1 * n1)) : 0};
        bool inb = true;
        for (int d = 0; d < 3; ++d) inb = inb && ijk[d] >= L.box.lo[d] && ijk[d] < L.box.lo[d] + L.box.dims[d];
        out[f] = inb ? (lab[L.box.idx(ijk[0], ijk[1], ijk[2])] & KIND_MASK) : 0;
    }
}

int iim_node_labels(const iim_problem* h, uint8_t* labels) {
    ABI_TRY({
        if (!h || !labels) throw Error(IIM_E_INVALID_ARG, "null argument");
        labels_to_full(*h->p, 0, labels);
        return IIM_OK;
    })
}

int iim_set_boundary_data(iim_problem* h, const double* cp_data, const double* box_data, int32_t mem_kind) {
    ABI_TRY({
        if (!h) throw Error(IIM_E_INVALID_ARG, "null argument");
        h->p->set_boundary_data(cp_data, box_data, mem_kind);
        return IIM_OK;
    })
}

int iim_set_boundary_data_noalloc(iim_problem* h, const double* cp_data, const double* box_data,
                                  int32_t mem_kind) {
    ABI_TRY({
        if (!h) throw Error(IIM_E_INVALID_ARG, "null argument");
        Problem& p = *h->p;
        double* staging = nullptr;
        if (box_data) {
            const int64_t n1 = p.grid.n + 1;
            const int64_t tot = p.dim == 2 ? n1 * n1 : n1 * n1 * n1;
            if (tot > IIM_NOALLOC_MAX_NODES)
                throw Error(IIM_E_INVALID_ARG, "box data of " + std::to_string(tot) +
                                                   " nodes exceed the static staging array (IIM_NOALLOC_MAX_NODES)");
            int dev = 0;
            IIM_HIP(hipGetDevice(&dev));
            if (dev != p.mem.device) throw Error(IIM_E_INVALID_ARG, "the handle's device is not the current one");
            staging = noalloc_scratch(dev);
        }
        p.set_boundary_data(cp_data, box_data, mem_kind, staging);
        return IIM_OK;
    })
}

int iim_set_rhs(iim_problem* h, const double* f, int32_t mem_kind) {
    ABI_TRY({
        if (!h) throw Error(IIM_E_INVALID_ARG, "null argument");
        h->p->set_rhs(f, mem_kind);
        return IIM_OK;
    })
}

int iim_solve(iim_problem* h, double* u, const double* x0, double* hist, int32_t hist_cap, iim_stats* st) {
    ABI_TRY({
        if (!h) throw Error(IIM_E_INVALID_ARG, "null argument");
        int r = h->p->solve(u, x0, hist, hist_cap, st);
        if (r == IIM_E_BREAKDOWN) iim::set_error("FGMRES breakdown (non-finite value)");
        if (r == IIM_NOT_CONVERGED) iim::set_error("FGMRES reached max_iters");
        return r;
    })
}

int iim_apply(iim_problem* h, const double* x, double* y, int32_t with_data) {
    ABI_TRY({
        if (!h || !x || !y) throw Error(IIM_E_INVALID_ARG, "null argument");
        Problem& p = *h->p;
        run_full_to_box(p.dim, p.grid.n, p.box, x, p.rk, p.levels[0].labels, 1, p.stream);
        p.apply_box(p.rk, p.wk, with_data);
        run_box_to_full(p.dim, p.grid.n, p.box, p.wk, p.levels[0].labels, 0.0, y, p.stream);
        IIM_HIP(hipStreamSynchronize(p.stream));
        return IIM_OK;
    })
}

int iim_vcycle(iim_problem* h, const double* v, double* z) {
    ABI_TRY({
        if (!h || !v || !z) throw Error(IIM_E_INVALID_ARG, "null argument");
        Problem& p = *h->p;
        run_full_to_box(p.dim, p.grid.n, p.box, v, p.rk, p.levels[0].labels, 1, p.stream);
        p.vcycle(p.rk, p.wk);
        run_box_to_full(p.dim, p.grid.n, p.box, p.wk, p.levels[0].labels, 0.0, z, p.stream);
        IIM_HIP(hipStreamSynchronize(p.stream));
        return IIM_OK;
    })
}

int iim_gradient(iim_problem* h, const double* u, double* grad) {
    ABI_TRY({
        if (h && h->p->grid.periodic) throw Error(IIM_E_INVALID_ARG, "no gradient post-processing on periodic grids");
        if (!h || !u || !grad) throw Error(IIM_E_INVALID_ARG, "null argument");
        Problem& p = *h->p;
        const int64_t n1 = p.grid.n + 1;
        const int64_t total = p.dim == 2 ? n1 * n1 : n1 * n1 * n1;
        run_fill(grad, p.dim * total, std::nan(""), p.stream);
        run_full_to_box(p.dim, p.grid.n, p.box, u, p.rk, p.levels[0].labels, 1, p.stream);
        run_ghosts(p.ghost_dev(), p.rk, p.cpdata, 1, p.ghost, p.stream);
        const Level& L0 = p.levels[0];
        run_ho_gradient(p.dim, p.box, L0.core_lo, L0.core_hi, p.grid.n, L0.labels, p.ho_irr_index, p.ho_slots, p.ghost,
                        p.boxval, p.w, 1.0 / p.h, p.rk, grad, p.stream);
        IIM_HIP(hipStreamSynchronize(p.stream));
        return IIM_OK;
    })
}

int iim_boundary_quantity(iim_problem* h, const double* u, double* q) {
    ABI_TRY({
        if (!h || !u || !q) throw Error(IIM_E_INVALID_ARG, "null argument");
        Problem& p = *h->p;
        p.ensure_normal_rows();
        run_full_to_box(p.dim, p.grid.n, p.box, u, p.rk, p.levels[0].labels, 1, p.stream);
        BQDev B;
        B.bc = p.bc;
        B.nsides = p.nsides;
        B.w = p.w;
        B.nrows = p.w + 1;
        B.beta_plus = p.opt.beta_plus;
        B.beta_minus = p.opt.beta_minus;
        const bool own = p.nrows == p.w + 1;  // the setup's fits already carry the row
        B.ptr = own ? p.ls_ptr : p.nd_ptr;
        B.idx = own ? p.ls_idx : p.nd_idx;
        B.Sd = own ? p.ls_S + (size_t)p.w * p.nnz : p.nd_S + (size_t)p.w * p.nd_nnz;
        B.Sc = own ? p.ls_Sc : p.nd_Sc;
        B.ncp = p.cp.ncp;
        run_boundary_quantity(B, p.rk, p.cpdata, q, p.stream);
        IIM_HIP(hipStreamSynchronize(p.stream));
        return IIM_OK;
    })
}

int iim_wall_gradient(iim_problem* h, const double* u, double* grad, const double* u_inf, double* cp) {
    ABI_TRY({
        if (!h || !u || !grad) throw Error(IIM_E_INVALID_ARG, "null argument");
        if ((u_inf == nullptr) != (cp == nullptr)) throw Error(IIM_E_INVALID_ARG, "u_inf and cp go together");
        Problem& p = *h->p;
        WGDev G{};
        if (u_inf) {
            double u2 = 0.0;
            for (int d = 0; d < p.dim; ++d) {
                G.u_inf[d] = u_inf[d];
                u2 += u_inf[d] * u_inf[d];
            }
            if (!(u2 > 0.0)) throw Error(IIM_E_INVALID_ARG, "u_inf must be non-zero");
        }
        p.ensure_grad_rows();
        run_full_to_box(p.dim, p.grid.n, p.box, u, p.rk, p.levels[0].labels, 1, p.stream);
        G.bc = p.bc;
        G.nsides = p.nsides;
        G.dim = p.dim;
        G.beta_plus = p.opt.beta_plus;
        G.beta_minus = p.opt.beta_minus;
        G.ptr = p.gd_ptr;
        G.idx = p.gd_idx;
        G.S = p.gd_S;
        G.Sc = p.gd_Sc;
        G.ncp = p.cp.ncp;
        run_wall_gradient(G, p.rk, p.cpdata, grad, cp, p.stream);
        IIM_HIP(hipStreamSynchronize(p.stream));
        return IIM_OK;
    })
}

int iim_ls_stencil(const iim_problem* h, int64_t c, int32_t side, int32_t* m, int32_t* r, int64_t* idx, double* wts,
                   int32_t cap) {
    ABI_TRY({
        if (!h || !m || !r) throw Error(IIM_E_INVALID_ARG, "null argument");
        const Problem& p = *h->p;
        if (c < 0 || c >= p.cp.ncp) throw Error(IIM_E_INVALID_ARG, "control point out of range");
        if (side != 1 && !(side == 2 && p.nsides == 2)) throw Error(IIM_E_INVALID_ARG, "bad side");
        const int64_t cs = c * p.nsides + (side == 1 ? 0 : 1);
        const int64_t b0 = p.h_ptr[cs], b1 = p.h_ptr[cs + 1];
        *m = (int32_t)(b1 - b0);
        *r = p.nrows;
        if (!idx && !wts) return IIM_OK;
        if (*m + 1 > cap) throw Error(IIM_E_INVALID_ARG, "capacity too small");
        std::vector<int32_t> li(b1 - b0);
        std::vector<double> sc(p.nrows), s((size_t)p.nrows * (b1 - b0));
        if (b1 > b0) IIM_HIP(hipMemcpyAsync(li.data(), p.ls_idx + b0, (b1 - b0) * sizeof(int32_t), hipMemcpyDeviceToHost, p.stream));
        IIM_HIP(hipMemcpyAsync(sc.data(), p.ls_Sc + cs * p.nrows, p.nrows * sizeof(double), hipMemcpyDeviceToHost, p.stream));
        for (int k = 0; k < p.nrows; ++k)
            if (b1 > b0)
                IIM_HIP(hipMemcpyAsync(s.data() + (size_t)k * (b1 - b0), p.ls_S + (size_t)k * p.nnz + b0,
                                       (b1 - b0) * sizeof(double), hipMemcpyDeviceToHost, p.stream));
        IIM_HIP(hipStreamSynchronize(p.stream));
        const int64_t n1 = p.grid.n + 1;
        for (int64_t a = 0; a < b1 - b0; ++a) {
            int ijk[3];
            p.box.coords(li[a], ijk);
            if (idx) idx[a] = ijk[0] + n1 * (ijk[1] + n1 * (int64_t)ijk[2]);
        }
        if (wts) {
            for (int k = 0; k < p.nrows; ++k) {
                wts[k] = sc[k];
                for (int64_t a = 0; a < b1 - b0; ++a) wts[(1 + a) * p.nrows + k] = s[(size_t)k * (b1 - b0) + a];
            }
        }
        return IIM_OK;
    })
}

int iim_level_info(const iim_problem* h, int32_t level, int32_t* n, int64_t* nunk) {
    ABI_TRY({
        if (!h) throw Error(IIM_E_INVALID_ARG, "null argument");
        const Problem& p = *h->p;
        if (level < 0 || level >= (int)p.levels.size()) throw Error(IIM_E_INVALID_ARG, "level out of range");
        if (n) *n = p.levels[level].n;
        if (nunk) *nunk = p.levels[level].nunk;
        return IIM_OK;
    })
}

int iim_level_labels(const iim_problem* h, int32_t level, uint8_t* labels) {
    ABI_TRY({
        if (!h || !labels) throw Error(IIM_E_INVALID_ARG, "null argument");
        const Problem& p = *h->p;
        if (level < 0 || level >= (int)p.levels.size()) throw Error(IIM_E_INVALID_ARG, "level out of range");
        labels_to_full(p, level, labels);
        return IIM_OK;
    })
}

int iim_level_op(iim_problem* h, int32_t level, int32_t op, const double* in1, double* out) {
    ABI_TRY({
        if (!h || !in1 || !out) throw Error(IIM_E_INVALID_ARG, "null argument");
        Problem& p = *h->p;
        return p.level_op(level, op, in1, out);
    })
}

int iim_time_kernel(iim_problem* h, int32_t kernel, int32_t reps, double* avg_ms) {
    ABI_TRY({
        if (!h || !avg_ms || reps < 1) throw Error(IIM_E_INVALID_ARG, "bad argument");
        Problem& p = *h->p;
        *avg_ms = p.time_kernel(kernel, reps);
        return IIM_OK;
    })
}

int iim_set_synthetic_data(iim_problem* h, int32_t kind) {
    ABI_TRY({
        if (!h) throw Error(IIM_E_INVALID_ARG, "null argument");
        h->p->synth_data(kind);
        IIM_HIP(hipStreamSynchronize(h->p->stream));
        return IIM_OK;
    })
}

int iim_synthetic_error(iim_problem* h, int32_t kind, const double* u, double* max_err) {
    ABI_TRY({
        if (!h || !u || !max_err) throw Error(IIM_E_INVALID_ARG, "null argument");
        *max_err = h->p->synth_error(kind, u);
        return IIM_OK;
    })
}

}  // extern "C"
