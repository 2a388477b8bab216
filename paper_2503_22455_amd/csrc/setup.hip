// Setup kernels: node labels, control points, irregular-node records and the
// Shortley-Weller hierarchy (Sec. 2.1 and 3.1-3.3 of the paper).
#include <mutex>

#include "kernels.h"

namespace iim {

// ---------------------------------------------------------------------------
// labels
// ---------------------------------------------------------------------------
// Pass 1, one launch for every level (blockIdx.y = level): each block
// classifies a grid-stride share of the level's nodes and writes its partial
// {min x,y,z, max x,y,z, touches-the-box flag, unknown count} to part.
// The two kernels below evaluate the level set at every node of a level, with
// the dimension as a template parameter (a runtime dimension turned every
// coordinate into a chain of selects) and a linear index below 2^31 split by
// 32-bit division (cfg-4 setup 27.9 -> 25.4 ms).  The parameters stay in
// global memory: read through the scalar cache they are free operands, and a
// copy in LDS made both kernels slower.
// node (i, j, k) of linear index l in an n1 x n1 (x n1) grid or a box
__device__ inline void split_index(int64_t l, int64_t d0, int64_t d1, bool narrow, int* ijk) {
    if (narrow) {
        const uint32_t l32 = (uint32_t)l, a = (uint32_t)d0, b = (uint32_t)d1;
        const uint32_t q = l32 / a;
        ijk[0] = (int)(l32 - q * a);
        ijk[1] = (int)(q % b);
        ijk[2] = (int)(q / b);
    } else {
        const int64_t q = l / d0;
        ijk[0] = (int)(l - q * d0);
        ijk[1] = (int)(q % d1);
        ijk[2] = (int)(q / d1);
    }
}

template <int DIM>
__device__ inline void classify_share(const Geom& g, const double* gp, int* mn, int* mx, int& cnt, int& bad) {
    const int64_t n1 = g.n + 1;
    const int64_t total = DIM == 2 ? n1 * n1 : n1 * n1 * n1;
    const bool narrow = total < ((int64_t)1 << 31);
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < total;
         l += (int64_t)gridDim.x * blockDim.x) {
        int ijk[3];
        split_index(l, n1, n1, narrow, ijk);
        if (DIM == 2) ijk[2] = 0;
        const uint8_t k = node_kind_d<DIM>(g, gp, ijk);
        if (k == 255) {
            bad = 1;
            continue;
        }
        if (k == K_PLUS || k == K_MINUS) {
            for (int d = 0; d < 3; ++d) {
                mn[d] = min(mn[d], ijk[d]);
                mx[d] = max(mx[d], ijk[d]);
            }
            ++cnt;
        }
    }
}

__global__ void __launch_bounds__(256) k_classify_levels(GeomSet G, int* part) {
    __shared__ int sh[8][256];
    const Geom& g = G.g[blockIdx.y];
    const double* gp = g.p;
    int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    int cnt = 0, bad = 0;
    if (g.dim == 3)
        classify_share<3>(g, gp, mn, mx, cnt, bad);
    else
        classify_share<2>(g, gp, mn, mx, cnt, bad);
    const int t = threadIdx.x;
    for (int d = 0; d < 3; ++d) {
        sh[d][t] = mn[d];
        sh[3 + d][t] = mx[d];
    }
    sh[6][t] = bad;
    sh[7][t] = cnt;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            for (int d = 0; d < 3; ++d) {
                sh[d][t] = min(sh[d][t], sh[d][t + off]);
                sh[3 + d][t] = max(sh[3 + d][t], sh[3 + d][t + off]);
            }
            sh[6][t] |= sh[6][t + off];
            sh[7][t] += sh[7][t + off];
        }
        __syncthreads();
    }
    if (t < 8) part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 8 + t] = sh[t][0];
}

// Pass 2, one block per level: bbox[8 l + 0..6] and count[l] from the partials
__global__ void __launch_bounds__(256) k_classify_reduce(const int* part, int nb, int* bbox,
                                                         unsigned long long* count) {
    __shared__ int sh[7][256];
    __shared__ unsigned long long shc[256];
    const int t = threadIdx.x;
    int v[7] = {1 << 30, 1 << 30, 1 << 30, -(1 << 30), -(1 << 30), -(1 << 30), 0};
    unsigned long long c = 0;
    for (int b = t; b < nb; b += blockDim.x) {
        const int* q = part + ((int64_t)blockIdx.x * nb + b) * 8;
        for (int d = 0; d < 3; ++d) {
            v[d] = min(v[d], q[d]);
            v[3 + d] = max(v[3 + d], q[3 + d]);
        }
        v[6] |= q[6];
        c += (unsigned long long)q[7];
    }
    for (int d = 0; d < 7; ++d) sh[d][t] = v[d];
    shc[t] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            for (int d = 0; d < 3; ++d) {
                sh[d][t] = min(sh[d][t], sh[d][t + off]);
                sh[3 + d][t] = max(sh[3 + d][t], sh[3 + d][t + off]);
            }
            sh[6][t] |= sh[6][t + off];
            shc[t] += shc[t + off];
        }
        __syncthreads();
    }
    if (t < 7) bbox[8 * blockIdx.x + t] = sh[t][0];
    if (t == 0) count[blockIdx.x] = shc[0];
}

int classify_part_ints(int nl) { return nl * CLASSIFY_BLOCKS * 8; }

void run_classify_levels(const GeomSet& G, int nl, int* d_part, int* d_bbox, unsigned long long* d_count,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_classify_levels, dim3(CLASSIFY_BLOCKS, nl), dim3(256), 0, s, G, d_part);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_classify_reduce, dim3(nl), dim3(256), 0, s, d_part, CLASSIFY_BLOCKS, d_bbox, d_count);
    IIM_LAUNCH_CHECK();
}

template <int DIM>
__device__ inline void box_labels_share(const Geom& g, const double* gp, const Box& b, uint8_t* labels) {
    const int64_t total = b.size();
    const bool narrow = total < ((int64_t)1 << 31);
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < total;
         l += (int64_t)gridDim.x * blockDim.x) {
        int ijk[3];
        split_index(l, b.dims[0], b.dims[1], narrow, ijk);
        for (int d = 0; d < 3; ++d) ijk[d] += b.lo[d];
        bool in = true;
        for (int d = 0; d < DIM; ++d) in = in && ijk[d] >= 0 && ijk[d] <= g.n;
        uint8_t k = in ? node_kind_d<DIM>(g, gp, ijk) : K_INACTIVE;
        labels[l] = (k == 255) ? K_INACTIVE : k;
    }
}

__global__ void __launch_bounds__(256) k_box_labels(LevelSet S) {
    const Geom& g = S.g[blockIdx.y];
    const double* gp = g.p;
    if (g.dim == 3)
        box_labels_share<3>(g, gp, S.b[blockIdx.y], S.labels[blockIdx.y]);
    else
        box_labels_share<2>(g, gp, S.b[blockIdx.y], S.labels[blockIdx.y]);
}

void run_box_labels(const LevelSet& S, int nl, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(cdiv(S.b[0].size(), 256), 4096);
    hipLaunchKernelGGL(k_box_labels, dim3(blocks, nl), dim3(256), 0, s, S);
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// control points
// ---------------------------------------------------------------------------
__device__ inline bool crossing_pair(uint8_t la, uint8_t lb, int side) {
    la &= KIND_MASK;
    lb &= KIND_MASK;
    if (side == IIM_SIDE_INTERFACE)
        return (la == K_PLUS && lb == K_MINUS) || (la == K_MINUS && lb == K_PLUS);
    return (la == K_PLUS && lb == K_INACTIVE) || (la == K_INACTIVE && lb == K_PLUS);
}

__global__ void k_cp_flags(Geom g, Box b, const uint8_t* labels, uint8_t* flags_all) {
    const int axis = blockIdx.y;
    int64_t total = b.size();
    int64_t st = b.stride(axis);
    uint8_t* flags = flags_all + axis * total;
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < total;
         l += (int64_t)gridDim.x * blockDim.x) {
        int ijk[3];
        b.coords(l, ijk);
        if (g.periodic) {
            // every segment, the last one of a line closing through the image of node 0
            const int64_t q = ijk[axis] + 1 < g.n ? l + st : l - (int64_t)(g.n - 1) * st;
            flags[l] = crossing_pair(labels[l], labels[q], g.side) ? 1 : 0;
            continue;
        }
        bool ok = ijk[axis] - b.lo[axis] + 1 < b.dims[axis];
        for (int d = 0; d < g.dim; ++d) ok = ok && ijk[d] >= 0 && ijk[d] <= g.n;
        ok = ok && ijk[axis] + 1 <= g.n;
        flags[l] = (ok && crossing_pair(labels[l], labels[l + st], g.side)) ? 1 : 0;
    }
}

void run_cp_flags(const Geom& g, const Box& b, const uint8_t* labels, uint8_t* flags, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(cdiv(b.size(), 256), 4096);
    hipLaunchKernelGGL(k_cp_flags, dim3(blocks, g.dim), dim3(256), 0, s, g, b, labels, flags);
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// flagged selections, several at once, in three launches: per-block counts,
// one scan per selection, an ordered scatter (ballot prefix within wavefronts)
// ---------------------------------------------------------------------------
constexpr int SEL_TILE = 16;
__device__ inline void sel_chunk(int64_t n, int b, int64_t* lo, int64_t* hi) {
    const int64_t c = (n + SEL_BLOCKS - 1) / SEL_BLOCKS;
    *lo = min(n, (int64_t)b * c);
    *hi = min(n, *lo + c);
}

__global__ void __launch_bounds__(256) k_sel_count(SelSet S, int* part) {
    __shared__ int sh[256];
    const SelItem& it = S.it[blockIdx.y];
    int64_t lo, hi;
    sel_chunk(it.n, blockIdx.x, &lo, &hi);
    // SEL_TILE consecutive flags per thread and step, their loads independent
    int c = 0;
    for (int64_t l0 = lo + SEL_TILE * (int64_t)threadIdx.x; l0 < hi; l0 += SEL_TILE * (int64_t)blockDim.x) {
        uint8_t v[SEL_TILE];
#pragma unroll
        for (int j = 0; j < SEL_TILE; ++j) v[j] = l0 + j < hi ? it.flags[l0 + j] : 0;
#pragma unroll
        for (int j = 0; j < SEL_TILE; ++j) c += v[j] != 0;
    }
    const int t = threadIdx.x;
    sh[t] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.y * SEL_BLOCKS + blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(SEL_BLOCKS) k_sel_scan(SelSet S, int* part) {
    __shared__ int sh[SEL_BLOCKS];
    int* p = part + blockIdx.x * SEL_BLOCKS;
    const int t = threadIdx.x;
    const int v = p[t];
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SEL_BLOCKS; off <<= 1) {
        const int a = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    p[t] = sh[t] - v;  // first output slot of block t
    if (t == SEL_BLOCKS - 1) *S.it[blockIdx.x].count = sh[t];
}

// the block's steps cover 256 x SEL_TILE consecutive flags: thread t takes
// the SEL_TILE flags from t0 + SEL_TILE t on and writes its selected indices
// after those of the threads before it (an exclusive scan of the per-thread
// counts), so the output keeps increasing index order
__global__ void __launch_bounds__(256) k_sel_scatter(SelSet S, const int* part) {
    __shared__ int wsum[4];
    const SelItem& it = S.it[blockIdx.y];
    int64_t lo, hi;
    sel_chunk(it.n, blockIdx.x, &lo, &hi);
    int base = part[blockIdx.y * SEL_BLOCKS + blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int64_t t0 = lo; t0 < hi; t0 += SEL_TILE * 256) {
        const int64_t l0 = t0 + SEL_TILE * (int64_t)t;
        uint8_t v[SEL_TILE];
#pragma unroll
        for (int j = 0; j < SEL_TILE; ++j) v[j] = l0 + j < hi ? it.flags[l0 + j] : 0;
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < SEL_TILE; ++j) cnt += v[j] != 0;
        int inc = cnt;  // inclusive scan over the wavefront
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(inc, d, 64);
            if (lane >= d) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int off = 0;
        for (int q = 0; q < w; ++q) off += wsum[q];
        const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        int pos = base + off + inc - cnt;
#pragma unroll
        for (int j = 0; j < SEL_TILE; ++j)
            if (v[j]) it.out[pos++] = (int32_t)(l0 + j);
        base += tot;
        __syncthreads();
    }
}

void select_flagged_multi(const SelItem* items, int k, int* d_part, hipStream_t s) {
    if (k < 1 || k > SEL_MAX) throw Error(IIM_E_INTERNAL, "selection count out of range");
    SelSet S{};
    for (int i = 0; i < k; ++i) {
        if (items[i].n < 0 || items[i].n > (int64_t)INT32_MAX) throw Error(IIM_E_INTERNAL, "selection too long");
        S.it[i] = items[i];
    }
    hipLaunchKernelGGL(k_sel_count, dim3(SEL_BLOCKS, k), dim3(256), 0, s, S, d_part);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_scan, dim3(k), dim3(SEL_BLOCKS), 0, s, S, d_part);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_scatter, dim3(SEL_BLOCKS, k), dim3(256), 0, s, S, (const int*)d_part);
    IIM_LAUNCH_CHECK();
}

__global__ void k_cp_compute(Geom g, Box b, const uint8_t* labels, CPDev cp, int* err) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cp.ncp) return;
    int axis = cp.axis[c];
    int64_t p = cp.lower[c];
    int pijk[3];
    b.coords(p, pijk);
    // upper node: on a periodic grid the last segment of a line closes through node 0
    int64_t q = (g.periodic && pijk[axis] == g.n - 1) ? p - (int64_t)(g.n - 1) * b.stride(axis) : p + b.stride(axis);
    uint8_t kp = labels[p] & KIND_MASK;
    int64_t a;
    if (g.side == IIM_SIDE_INTERFACE)
        a = (kp == K_MINUS) ? p : q;
    else
        a = (kp == K_PLUS) ? p : q;
    int dir = (a == p) ? 1 : -1;
    // coordinates of the root-search node; on a periodic grid unwrapped: q sits
    // at x_p + h e_axis
    double xa[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < g.dim; ++d) xa[d] = node_coord(g, pijk[d]);
    if (a == q) xa[axis] = g.periodic ? node_coord(g, pijk[axis]) + g.h : node_coord(g, pijk[axis] + 1);
    int which = 0;
    double root = crossing_root(g, xa, axis, dir, &which);
    double x[3] = {xa[0], xa[1], xa[2]};
    x[axis] = root;
    double nv[3];
    geom_normal(g, x, which, nv);
    double kap = geom_curvature(g, x, which);
    for (int d = 0; d < 3; ++d) {
        cp.x[d * cp.ncp + c] = x[d];
        cp.n[d * cp.ncp + c] = nv[d];
    }
    cp.kappa[c] = kap;
    // side 0 = Omega^+, side 1 = Omega^-
    int64_t aplus = (kp == K_PLUS) ? p : q;
    cp.a[c] = (int32_t)aplus;
    cp.dir[c] = (aplus == p) ? 1 : -1;
    if (cp.nsides == 2) {
        int64_t aminus = (kp == K_MINUS) ? p : q;
        cp.a[cp.ncp + c] = (int32_t)aminus;
        cp.dir[cp.ncp + c] = (aminus == p) ? 1 : -1;
    }
    if (!(fabs(kap * g.h) < 0.25)) atomicOr(err, 2);
}

void run_cp_compute(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp, int* d_err,
                    hipStream_t s) {
    if (cp.ncp == 0) return;
    hipLaunchKernelGGL(k_cp_compute, dim3(cdiv(cp.ncp, 128)), dim3(128), 0, s, g, b, labels, cp, d_err);
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// irregular high-order nodes
// ---------------------------------------------------------------------------
// index of the control point on segment (lower, lower + e_axis), -1 if none
__device__ inline int64_t find_cp(const CPDev& cp, int axis, int32_t lower) {
    int lo = cp.axis_start[axis], hi = cp.axis_start[axis + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int32_t v = cp.lower[mid];
        if (v == lower) return mid;
        if (v < lower) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// kind of node ijk + j dir e_d, or INACTIVE outside the grid; *l = its box index
__device__ inline uint8_t kind_at(const Geom& g, const Box& b, const uint8_t* labels, const int* ijk, int d,
                                  int step, int64_t* l) {
    int c[3] = {ijk[0], ijk[1], ijk[2]};
    c[d] += step;
    if (g.periodic) c[d] = wrap_index(c[d], g.n);
    if (c[d] < 0 || c[d] > g.n || c[d] < b.lo[d] || c[d] >= b.lo[d] + b.dims[d]) {
        *l = -1;
        return 255;
    }
    *l = b.idx(c[0], c[1], c[2]);
    return labels[*l] & KIND_MASK;
}

// true if a node of kind k at l (coordinates ijk) sees, within w nodes along
// an axis, a node of another kind or the edge of the box or grid (as kind_at,
// with the neighbour's index stepped from l along the axis)
template <int DIM>
__device__ inline bool ho_irregular_node(const Geom& g, const Box& b, const uint8_t* labels, int64_t l,
                                         const int* ijk, uint8_t k, int w) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int64_t st = b.stride(d);
        for (int s = -w; s <= w; ++s) {
            if (s == 0) continue;
            int c = ijk[d] + s;
            if (g.periodic) c = wrap_index(c, g.n);
            if (c < 0 || c > g.n || c < b.lo[d] || c >= b.lo[d] + b.dims[d]) return true;
            if ((labels[l + (int64_t)(c - ijk[d]) * st] & KIND_MASK) != k) return true;
        }
    }
    return false;
}

__global__ void k_ho_irr_flag(Geom g, Box b, uint8_t* labels, uint8_t* flags, int w) {
    int64_t total = b.size();
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < total;
         l += (int64_t)gridDim.x * blockDim.x) {
        uint8_t lab = labels[l];
        uint8_t k = lab & KIND_MASK;
        bool irr = false;
        if (k == K_PLUS || k == K_MINUS) {
            int ijk[3];
            b.coords(l, ijk);
            irr = g.dim == 3 ? ho_irregular_node<3>(g, b, labels, l, ijk, k, w)
                             : ho_irregular_node<2>(g, b, labels, l, ijk, k, w);
        }
        flags[l] = irr ? 1 : 0;
        if (irr) labels[l] = lab | F_HO_IRR;
    }
}

void run_ho_irr_flag(const Geom& g, const Box& b, uint8_t* labels, uint8_t* flags, int w, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(cdiv(b.size(), 256), 8192);
    hipLaunchKernelGGL(k_ho_irr_flag, dim3(blocks), dim3(256), 0, s, g, b, labels, flags, w);
    IIM_LAUNCH_CHECK();
}

// One record per irregular node: 2*dim slots, slot (d, dir) at 2d + (dir > 0).
__global__ void k_ho_irr_records(Geom g, Box b, const uint8_t* labels, CPDev cp, const int32_t* nodes,
                                 int64_t nirr, int32_t* slots, int32_t* irr_index, int w, int* err) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nirr) return;
    int64_t l = nodes[k];
    irr_index[l] = (int32_t)k;
    uint8_t side = labels[l] & KIND_MASK;
    int sidx = (side == K_PLUS) ? 0 : 1;
    int ijk[3];
    b.coords(l, ijk);
    for (int d = 0; d < g.dim; ++d)
        for (int t = 0; t < 2; ++t) {
            int dir = t ? 1 : -1;
            int slot = make_slot(SLOT_REG, 0, 0);
            int64_t prev = l;
            for (int j = 1; j <= w; ++j) {
                int64_t q;
                uint8_t kq = kind_at(g, b, labels, ijk, d, dir * j, &q);
                if (kq == side) {
                    prev = q;
                    continue;
                }
                if (kq == K_BOX) {
                    slot = make_slot(SLOT_BOX, j, 0);
                } else if (kq == 255) {
                    atomicOr(err, 4);  // stencil leaves the storage box
                } else {
                    // the segment's lower node: the one whose +e_d neighbour is the other
                    int64_t lower = dir > 0 ? prev : q;
                    int64_t c = find_cp(cp, d, (int32_t)lower);
                    if (c < 0) {
                        atomicOr(err, 8);
                    } else {
                        slot = make_slot(SLOT_GHOST, j, (int)(c * cp.nsides + sidx));
                    }
                }
                break;
            }
            slots[k * 2 * g.dim + 2 * d + t] = slot;
        }
}

void run_ho_irr_records(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp,
                        const int32_t* nodes, int64_t nirr, int32_t* slots, int32_t* irr_index, int w, int* d_err,
                        hipStream_t s) {
    if (nirr == 0) return;
    hipLaunchKernelGGL(k_ho_irr_records, dim3(cdiv(nirr, 128)), dim3(128), 0, s, g, b, labels, cp, nodes, nirr,
                       slots, irr_index, w, d_err);
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Shortley-Weller rows
// ---------------------------------------------------------------------------
__global__ void k_sw_irr_flag(LevelSet S, uint8_t* flags_all) {
    const Geom& g = S.g[blockIdx.y];
    const Box& b = S.b[blockIdx.y];
    uint8_t* labels = S.labels[blockIdx.y];
    uint8_t* flags = flags_all + S.off[blockIdx.y];
    int64_t total = b.size();
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < total;
         l += (int64_t)gridDim.x * blockDim.x) {
        uint8_t lab = labels[l];
        uint8_t k = lab & KIND_MASK;
        bool irr = false;
        if (k == K_PLUS || k == K_MINUS) {
            int ijk[3];
            b.coords(l, ijk);
            for (int d = 0; d < g.dim; ++d)
                for (int s = -1; s <= 1; s += 2) {
                    int64_t q;
                    uint8_t kq = kind_at(g, b, labels, ijk, d, s, &q);
                    if (kq != k && kq != K_BOX) irr = true;
                }
        }
        flags[l] = irr ? 1 : 0;
        if (irr) labels[l] = lab | F_SW_IRR;
    }
}

void run_sw_irr_flag(const LevelSet& S, int nl, uint8_t* flags, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(cdiv(S.b[0].size(), 256), 4096);
    hipLaunchKernelGGL(k_sw_irr_flag, dim3(blocks, nl), dim3(256), 0, s, S, flags);
    IIM_LAUNCH_CHECK();
}

// 1D row of the Shortley-Weller stencil, coefficients in units of 1/h^2.
// Side types: 0 = value (regular neighbour, Dirichlet or interface wall), 1 = Neumann wall.
__device__ inline void sw_row_1d(int tl, double pl, int tr, double pr, double* cl, double* cc, double* cr) {
    if (tl == 0 && tr == 0) {
        *cl = 2.0 / (pl * (pl + pr));
        *cc = -2.0 / (pl * pr);
        *cr = 2.0 / (pr * (pl + pr));
    } else if (tl == 1 && tr == 0) {
        double c = 2.0 / (pr * (2.0 * pl + pr));
        *cl = 0.0;
        *cc = -c;
        *cr = c;
    } else if (tl == 0 && tr == 1) {
        double c = 2.0 / (pl * (pl + 2.0 * pr));
        *cl = c;
        *cc = -c;
        *cr = 0.0;
    } else {
        *cl = *cc = *cr = 0.0;
    }
}

__global__ void k_sw_records(Geom g, Box b, const uint8_t* labels, const int32_t* nodes, int64_t nirr, int bc,
                             double beta_plus, double beta_minus, double* rec64, float* rec32,
                             int32_t* irr_index) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nirr) return;
    int64_t l = nodes[k];
    irr_index[l] = (int32_t)k;
    uint8_t kf = labels[l] & KIND_MASK;
    int ijk[3];
    b.coords(l, ijk);
    double xf[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < g.dim; ++d) xf[d] = node_coord(g, ijk[d]);
    const int R = 1 + 2 * g.dim;
    double row[7] = {0, 0, 0, 0, 0, 0, 0};
    double ap = 0.5 / beta_plus, am = 0.5 / beta_minus;
    for (int d = 0; d < g.dim; ++d) {
        int type[2];
        double psi[2], wself[2], wnb[2];
        for (int t = 0; t < 2; ++t) {
            int s = t ? 1 : -1;
            int64_t q;
            uint8_t kq = kind_at(g, b, labels, ijk, d, s, &q);
            type[t] = 0;
            psi[t] = 1.0;
            wself[t] = 0.0;
            wnb[t] = 0.0;
            if (kq == kf) {
                wnb[t] = 1.0;
            } else if (kq == K_BOX) {
                // known (zero) value at psi = 1
            } else if (g.side == IIM_SIDE_INTERFACE) {
                psi[t] = 0.5;
                // u_w = (alpha^+ u_minus + alpha^- u_plus) / (alpha^+ + alpha^-)
                double wm = ap / (ap + am), wp = am / (ap + am);
                wself[t] = (kf == K_MINUS) ? wm : wp;
                wnb[t] = (kf == K_MINUS) ? wp : wm;
            } else {
                int which;
                double root = crossing_root(g, xf, d, s, &which);
                double ps = fabs(root - xf[d]) / g.h;
                psi[t] = fmax(ps, 0.5);
                type[t] = (bc == IIM_BC_NEUMANN) ? 1 : 0;
            }
        }
        double cl, cc, cr;
        sw_row_1d(type[0], psi[0], type[1], psi[1], &cl, &cc, &cr);
        row[0] += cc + cl * wself[0] + cr * wself[1];
        row[1 + 2 * d] += cl * wnb[0];
        row[2 + 2 * d] += cr * wnb[1];
    }
    for (int r = 0; r < R; ++r) {
        rec64[k * R + r] = row[r];
        rec32[k * R + r] = (float)row[r];
    }
}

void run_sw_records(const Geom& g, const Box& b, const uint8_t* labels, const int32_t* nodes, int64_t nirr,
                    int bc, double beta_plus, double beta_minus, double* rec64, float* rec32, int32_t* irr_index,
                    hipStream_t s) {
    if (nirr == 0) return;
    hipLaunchKernelGGL(k_sw_records, dim3(cdiv(nirr, 128)), dim3(128), 0, s, g, b, labels, nodes, nirr, bc,
                       beta_plus, beta_minus, rec64, rec32, irr_index);
    IIM_LAUNCH_CHECK();
}

__global__ void k_fill_int(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void run_fill_int(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n == 0) return;
    int blocks = (int)std::min<int64_t>(cdiv(n, 256), 8192);
    hipLaunchKernelGGL(k_fill_int, dim3(blocks), dim3(256), 0, s, p, n, v);
    IIM_LAUNCH_CHECK();
}

// dense coarse matrix: row r of the listed unknowns; col_of[l] = column of box node l (-1 if excluded)
__global__ void k_coarse_assemble(Box b, int dim, int periodic, const uint8_t* labels, const int32_t* irr_index,
                                  const double* rec64, const int32_t* list, const int32_t* col_of, int64_t nc,
                                  double* A) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nc) return;
    int64_t l = list[r];
    for (int64_t c = 0; c < nc; ++c) A[r * nc + c] = 0.0;
    const int R = 1 + 2 * dim;
    bool irr = labels[l] & F_SW_IRR;
    double diag = irr ? rec64[irr_index[l] * R] : -2.0 * dim;
    A[r * nc + r] = diag;
    for (int d = 0; d < dim; ++d)
        for (int t = 0; t < 2; ++t) {
            int64_t q = l + (t ? 1 : -1) * b.stride(d);
            if (periodic) {  // the box is the periodic cell: neighbours modulo its width
                int ijk[3];
                b.coords(l, ijk);
                const int i2 = wrap_index(ijk[d] - b.lo[d] + (t ? 1 : -1), b.dims[d]);
                q = l + (int64_t)(i2 - (ijk[d] - b.lo[d])) * b.stride(d);
            }
            double c = irr ? rec64[irr_index[l] * R + 1 + 2 * d + t] : 1.0;
            int32_t col = col_of[q];
            if (c != 0.0 && col >= 0) A[r * nc + col] += c;
        }
}

void run_coarse_assemble(const Box& b, int dim, int periodic, const uint8_t* labels, const int32_t* irr_index,
                         const double* rec64, const int32_t* list, const int32_t* col_of, int64_t nc, double* A,
                         hipStream_t s) {
    if (nc == 0) return;
    hipLaunchKernelGGL(k_coarse_assemble, dim3(cdiv(nc, 64)), dim3(64), 0, s, b, dim, periodic, labels, irr_index,
                       rec64, list, col_of, nc, A);
    IIM_LAUNCH_CHECK();
}

// Gauss-Jordan inversion with partial pivoting, one workgroup (nc <= a few hundred).
__global__ void __launch_bounds__(1024) k_coarse_invert(double* A, double* X, int64_t nc, int* err) {
    __shared__ double red_v[1024];
    __shared__ int red_i[1024];
    __shared__ int piv_s;
    int tid = threadIdx.x;
    for (int64_t r = tid >> 6; r < nc; r += blockDim.x >> 6)
        for (int64_t c = tid & 63; c < nc; c += 64) X[r * nc + c] = r == c ? 1.0 : 0.0;
    __syncthreads();
    for (int64_t k = 0; k < nc; ++k) {
        double best = -1.0;
        int bi = -1;
        for (int64_t r = k + tid; r < nc; r += blockDim.x) {
            double v = fabs(A[r * nc + k]);
            if (v > best) {
                best = v;
                bi = (int)r;
            }
        }
        red_v[tid] = best;
        red_i[tid] = bi;
        __syncthreads();
        for (int off = blockDim.x / 2; off > 0; off >>= 1) {
            if (tid < off) {
                double v2 = red_v[tid + off];
                int i2 = red_i[tid + off];
                if (v2 > red_v[tid] || (v2 == red_v[tid] && i2 >= 0 && (red_i[tid] < 0 || i2 < red_i[tid]))) {
                    red_v[tid] = v2;
                    red_i[tid] = i2;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            piv_s = red_i[0];
            if (red_i[0] < 0 || red_v[0] == 0.0) atomicOr(err, 16);
        }
        __syncthreads();
        int piv = piv_s;
        if (piv < 0) return;
        if (piv != k) {
            for (int64_t c = tid; c < nc; c += blockDim.x) {
                double t = A[k * nc + c];
                A[k * nc + c] = A[piv * nc + c];
                A[piv * nc + c] = t;
                t = X[k * nc + c];
                X[k * nc + c] = X[piv * nc + c];
                X[piv * nc + c] = t;
            }
        }
        __syncthreads();
        double inv = 1.0 / A[k * nc + k];
        __syncthreads();
        for (int64_t c = tid; c < nc; c += blockDim.x) {
            A[k * nc + c] *= inv;
            X[k * nc + c] *= inv;
        }
        __syncthreads();
        // rows over wavefronts, columns over lanes (no index division per entry)
        for (int64_t r = tid >> 6; r < nc; r += blockDim.x >> 6) {
            if (r == k) continue;
            const double f = A[r * nc + k];
            for (int64_t c = tid & 63; c < nc; c += 64) {
                if (c == k) continue;  // column k of A updated last
                A[r * nc + c] -= f * A[k * nc + c];
                X[r * nc + c] -= f * X[k * nc + c];
            }
        }
        __syncthreads();
        for (int64_t r = tid; r < nc; r += blockDim.x) {
            if (r == k) continue;
            double f = A[r * nc + k];
            X[r * nc + k] -= f * X[k * nc + k];
            A[r * nc + k] = 0.0;
        }
        __syncthreads();
    }
}

// The same elimination with A and X resident in LDS (nc <= COARSE_LDS_NC): the
// steps, pivots and arithmetic of k_coarse_invert, without a device-memory round
// trip per step; the pivot search runs in one wavefront.
constexpr int COARSE_LDS_NC = 90;
__global__ void __launch_bounds__(1024) k_coarse_invert_lds(double* Ag, double* Xg, int nc, int* err) {
    extern __shared__ double lds[];
    double* A = lds;
    double* X = lds + nc * nc;
    __shared__ int piv_s;
    const int tid = threadIdx.x, n2 = nc * nc;
    for (int i = tid; i < n2; i += blockDim.x) {
        A[i] = Ag[i];
        X[i] = (i / nc == i % nc) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
        if (tid < 64) {
            double best = -1.0;
            int bi = -1;
            for (int r = k + tid; r < nc; r += 64) {
                const double v = fabs(A[r * nc + k]);
                if (v > best) {
                    best = v;
                    bi = r;
                }
            }
            // largest magnitude, the smallest row among equals
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double v2 = __shfl_xor(best, off, 64);
                const int i2 = __shfl_xor(bi, off, 64);
                if (v2 > best || (v2 == best && i2 >= 0 && (bi < 0 || i2 < bi))) {
                    best = v2;
                    bi = i2;
                }
            }
            if (tid == 0) {
                piv_s = bi;
                if (bi < 0 || best == 0.0) atomicOr(err, 16);
            }
        }
        __syncthreads();
        const int piv = piv_s;
        if (piv < 0) break;
        if (piv != k) {
            for (int c = tid; c < nc; c += blockDim.x) {
                double t = A[k * nc + c];
                A[k * nc + c] = A[piv * nc + c];
                A[piv * nc + c] = t;
                t = X[k * nc + c];
                X[k * nc + c] = X[piv * nc + c];
                X[piv * nc + c] = t;
            }
            __syncthreads();
        }
        const double inv = 1.0 / A[k * nc + k];
        __syncthreads();
        for (int c = tid; c < nc; c += blockDim.x) {
            A[k * nc + c] *= inv;
            X[k * nc + c] *= inv;
        }
        __syncthreads();
        for (int r = tid >> 6; r < nc; r += blockDim.x >> 6) {
            if (r == k) continue;
            const double f = A[r * nc + k];
            for (int c = tid & 63; c < nc; c += 64) {
                if (c == k) continue;  // column k of A updated last
                A[r * nc + c] -= f * A[k * nc + c];
                X[r * nc + c] -= f * X[k * nc + c];
            }
        }
        __syncthreads();
        for (int r = tid; r < nc; r += blockDim.x) {
            if (r == k) continue;
            const double f = A[r * nc + k];
            X[r * nc + k] -= f * X[k * nc + k];
            A[r * nc + k] = 0.0;
        }
        __syncthreads();
    }
    for (int i = tid; i < n2; i += blockDim.x) Xg[i] = X[i];
}

void run_coarse_invert(double* A, double* Ainv, int64_t nc, int* d_err, hipStream_t s) {
    if (nc == 0) return;
    if (nc <= COARSE_LDS_NC) {
        static std::once_flag once;
        std::call_once(once, [] {
            IIM_HIP(hipFuncSetAttribute((const void*)k_coarse_invert_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        2 * COARSE_LDS_NC * COARSE_LDS_NC * (int)sizeof(double)));
        });
        hipLaunchKernelGGL(k_coarse_invert_lds, dim3(1), dim3(1024), 2 * nc * nc * sizeof(double), s, A, Ainv, (int)nc,
                           d_err);
        IIM_LAUNCH_CHECK();
        return;
    }
    hipLaunchKernelGGL(k_coarse_invert, dim3(1), dim3(1024), 0, s, A, Ainv, nc, d_err);
    IIM_LAUNCH_CHECK();
}

}  // namespace iim
