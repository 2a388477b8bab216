// Hot-path operators: ghost values and the high-order apply (Sec. 2.1-2.3),
// and the Shortley-Weller V-cycle kernels (Sec. 3.1, 3.3).
//
// Storage: every level keeps its vectors in a padded bounding box of its
// unknowns (x fastest); nodes that are not unknowns hold zero, so regular
// stencils need no masks.  Nodes whose stencil differs from the constant one
// carry a flag in their label byte and an index into a compact record list.
#include <mutex>

#include "kernels.h"

namespace iim {

// ---------------------------------------------------------------------------
// ghost values: one group of GLN lanes per control point (all its sides); the
// group width follows the mean least-squares set size (16 lanes in 2D, a whole
// wavefront for the ~200-point 3D sets), rows and sides are compile-time
// ---------------------------------------------------------------------------
template <int NS, int NR, int GLN>
__global__ void __launch_bounds__(256) k_ghosts(GhostDev G, const double* __restrict__ x,
                                                const double* __restrict__ cpdata, int with_data,
                                                double* __restrict__ ghost) {
    const int lane = threadIdx.x % GLN;
    const int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / GLN;
    if (c >= G.ncp) return;  // whole groups exit together
    double dots[NS][NR];
#pragma unroll
    for (int sd = 0; sd < NS; ++sd) {
        const int64_t cs = c * NS + sd;
        const int64_t b0 = G.ptr[cs], b1 = G.ptr[cs + 1];
        double acc[2][NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[0][k] = acc[1][k] = 0.0;
        // GU entries per lane and step: all their index loads, then all their
        // gathers and weight loads are in flight together (a 3D set of ~235
        // points is one step: one index-then-gather round trip)
        constexpr int GU = 4;
        for (int64_t a0 = b0 + lane; a0 < b1; a0 += GU * GLN) {
            int32_t iv[GU];
#pragma unroll
            for (int u = 0; u < GU; ++u) iv[u] = a0 + u * GLN < b1 ? G.idx[a0 + u * GLN] : -1;
            double xv[GU];
#pragma unroll
            for (int u = 0; u < GU; ++u) xv[u] = iv[u] >= 0 ? x[iv[u]] : 0.0;
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int64_t a = a0 + u * GLN;
                if (a < b1)
#pragma unroll
                    for (int k = 0; k < NR; ++k) acc[u & 1][k] += G.W[k * G.nnz + a] * xv[u];
            }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            double v = acc[0][k] + acc[1][k];
#pragma unroll
            for (int off = GLN / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, GLN);
            dots[sd][k] = v;
        }
    }
    if (lane != 0) return;
    const int w = G.w;
    if (NS == 1) {
        for (int j = 0; j < w; ++j) {
            double gv = dots[0][j];
            if (with_data) gv += G.dcoef[c * w + j] * cpdata[c];
            ghost[c * w + j] = gv;
        }
        return;
    }
    // interface: Sec. 2.2 closed form with D = beta+ s_c+ - beta- s_c-
    const double* scp = G.Sc + (c * 2 + 0) * NR;
    const double* scm = G.Sc + (c * 2 + 1) * NR;
    const double bp = G.beta_plus, bm = G.beta_minus;
    const double D = bp * scp[w] - bm * scm[w];
    const double ubar = -(bp * dots[0][w] - bm * dots[NS - 1][w]) / D;
    double Up = ubar, Um = ubar;
    if (with_data) {
        const double j0 = cpdata[2 * c], j1 = cpdata[2 * c + 1];
        Up += (j1 - bm * scm[w] * j0) / D;
        Um += (j1 - bp * scp[w] * j0) / D;
    }
    for (int j = 0; j < w; ++j) {
        ghost[(c * 2 + 0) * w + j] = scp[j] * Up + dots[0][j];
        ghost[(c * 2 + 1) * w + j] = scm[j] * Um + dots[NS - 1][j];
    }
}

template <int NS, int NR>
static void launch_ghosts(const GhostDev& G, const double* x, const double* cpdata, int with_data, double* ghost,
                          hipStream_t s) {
    const double mean_m = (double)G.nnz / (double)(G.ncp * NS);
    const int gln = mean_m > 96.0 ? 64 : (mean_m > 40.0 ? 32 : 16);
    const int64_t threads = G.ncp * gln;
    if (gln == 64)
        hipLaunchKernelGGL((k_ghosts<NS, NR, 64>), dim3(cdiv(threads, 256)), dim3(256), 0, s, G, x, cpdata, with_data,
                           ghost);
    else if (gln == 32)
        hipLaunchKernelGGL((k_ghosts<NS, NR, 32>), dim3(cdiv(threads, 256)), dim3(256), 0, s, G, x, cpdata, with_data,
                           ghost);
    else
        hipLaunchKernelGGL((k_ghosts<NS, NR, 16>), dim3(cdiv(threads, 256)), dim3(256), 0, s, G, x, cpdata, with_data,
                           ghost);
    IIM_LAUNCH_CHECK();
}

void run_ghosts(const GhostDev& G, const double* x, const double* cpdata, int with_data, double* ghost,
                hipStream_t s) {
    if (G.ncp == 0) return;
    // rows: w ghosts (one side), w ghosts + the normal derivative (interfaces)
    if (G.nsides == 1 && G.nrows == G.w && G.w == 2)
        launch_ghosts<1, 2>(G, x, cpdata, with_data, ghost, s);
    else if (G.nsides == 2 && G.nrows == G.w + 1 && G.w == 2)
        launch_ghosts<2, 3>(G, x, cpdata, with_data, ghost, s);
    else if (G.nsides == 1 && G.nrows == G.w && G.w == 3)
        launch_ghosts<1, 3>(G, x, cpdata, with_data, ghost, s);
    else if (G.nsides == 2 && G.nrows == G.w + 1 && G.w == 3)
        launch_ghosts<2, 4>(G, x, cpdata, with_data, ghost, s);
    else
        throw Error(IIM_E_INTERNAL, "ghost kernel: unsupported rows/sides");
}

// ---------------------------------------------------------------------------
// high-order apply: y = beta/h^2 sum_d sum_j a_|j| u~(i + j e_d)
// ---------------------------------------------------------------------------
// values u~(l + jj sd), jj = 1..W, of the extended function along one half-line
// of an irregular node (label flag F_HO_IRR), from its slot record: grid values
// up to the first crossing, then ghost values (or box data with extrapolation
// past a box face)
template <int W>
__device__ inline void ho_half_line(int64_t l, int64_t sd, int slot, uint8_t kind,
                                    const uint8_t* __restrict__ labels, const double* __restrict__ ghost,
                                    const double* __restrict__ boxval, const double* __restrict__ x, int with_data,
                                    double (&v)[W]) {
    const int type = slot_type(slot), j0 = slot_j(slot);
    for (int jj = 1; jj <= W; ++jj) {
        const int64_t q = l + jj * sd;
        double val;
        if (type == SLOT_REG || jj < j0) {
            val = x[q];
        } else if (type == SLOT_GHOST) {
            uint8_t kq = labels[q] & KIND_MASK;
            if (kq == kind)
                val = x[q];  // back on the stencil's side beyond a sliver
            else if (kq == K_BOX)
                val = with_data ? boxval[q] : 0.0;
            else
                val = ghost[(int64_t)slot_cs(slot) * W + (jj - j0)];
        } else {  // box face at offset j0
            const int64_t face = l + j0 * sd;
            const double fv = with_data ? boxval[face] : 0.0;
            if (jj == j0) {
                val = fv;
            } else {
                // degree-2W Lagrange extrapolation jj - j0 steps beyond the face
                const int sb = jj - j0;
                val = ho_ext<W>(sb, 0) * fv;
#pragma unroll
                for (int u = 1; u <= 2 * W; ++u) val += ho_ext<W>(sb, u) * x[face - u * sd];
            }
        }
        v[jj - 1] = val;
    }
}

// contribution of the off-centre points of an irregular node
template <int DIM, int W>
__device__ inline double ho_irregular(const Box& b, int64_t l, uint8_t kind, const uint8_t* __restrict__ labels,
                                      const int32_t* __restrict__ rec, const double* __restrict__ ghost,
                                      const double* __restrict__ boxval, const double* __restrict__ x,
                                      int with_data) {
    const int64_t st[3] = {1, (int64_t)b.dims[0], (int64_t)b.dims[0] * b.dims[1]};
    double acc = 0.0;
    for (int d = 0; d < DIM; ++d)
        for (int t = 0; t < 2; ++t) {
            const int dir = t ? 1 : -1;
            double v[W];
            ho_half_line<W>(l, dir * st[d], rec[2 * d + t], kind, labels, ghost, boxval, x, with_data, v);
            double tw = ho_a<W>(1) * v[0] + ho_a<W>(2) * v[1];
            if (W == 3) tw += ho_a<W>(3) * v[W - 1];
            acc += tw;
        }
    return acc;
}

template <int DIM, int W>
__global__ void __launch_bounds__(256) k_ho_apply(Box b, int3 clo, int3 chi, const uint8_t* __restrict__ labels,
                                                  const int32_t* __restrict__ irr_index,
                                                  const int32_t* __restrict__ slots, const double* __restrict__ ghost,
                                                  const double* __restrict__ boxval, double inv_h2, double bp,
                                                  double bm, const double* __restrict__ x, double* __restrict__ y,
                                                  int with_data) {
    int i = clo.x + blockIdx.x * blockDim.x + threadIdx.x;
    int j = clo.y + blockIdx.y * blockDim.y + threadIdx.y;
    int k = DIM == 3 ? clo.z + blockIdx.z : 0;
    if (i > chi.x || j > chi.y) return;
    const int64_t l = b.idx(i, j, k);
    const uint8_t lab = labels[l];
    const uint8_t kind = lab & KIND_MASK;
    if (kind != K_PLUS && kind != K_MINUS) {
        y[l] = 0.0;
        return;
    }
    const double beta = (kind == K_PLUS) ? bp : bm;
    const int64_t st[3] = {1, (int64_t)b.dims[0], (int64_t)b.dims[0] * b.dims[1]};
    const double xc = x[l];
    double acc = (double)DIM * ho_a<W>(0) * xc;
    if (!(lab & F_HO_IRR)) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double tw = ho_a<W>(1) * (x[l + st[d]] + x[l - st[d]]) + ho_a<W>(2) * (x[l + 2 * st[d]] + x[l - 2 * st[d]]);
            if (W == 3) tw += ho_a<W>(3) * (x[l + 3 * st[d]] + x[l - 3 * st[d]]);
            acc += tw;
        }
        y[l] = beta * inv_h2 * acc;
        return;
    }
    acc += ho_irregular<DIM, W>(b, l, kind, labels, slots + (int64_t)irr_index[l] * 2 * DIM, ghost, boxval, x,
                                with_data);
    y[l] = beta * inv_h2 * acc;
}

// Apply on a periodic grid whose storage box is the periodic cell: one thread
// per node, neighbours modulo n, irregular half-lines from their slots (grid
// values up to the first crossing, then ghost values; a point back on the
// stencil's side beyond a sliver reads the grid).  (4,5) scheme.
template <int DIM>
__device__ inline double ho_periodic_node(const Box& b, int n, int64_t l, uint8_t lab,
                                          const int32_t* __restrict__ irr_index, const int32_t* __restrict__ slots,
                                          const uint8_t* __restrict__ labels, const double* __restrict__ ghost,
                                          double inv_h2, double bp, double bm, const double* __restrict__ x) {
    constexpr int W = 2;
    const uint8_t kind = lab & KIND_MASK;
    int ijk[3];
    b.coords(l, ijk);
    const int64_t st[3] = {1, (int64_t)b.dims[0], (int64_t)b.dims[0] * b.dims[1]};  // the box is the cell: dims n
    const bool irr = lab & F_HO_IRR;
    const int32_t* rec = irr ? slots + (int64_t)irr_index[l] * 2 * DIM : nullptr;
    double acc = (double)DIM * ho_a<W>(0) * x[l];
    for (int d = 0; d < DIM; ++d)
        for (int t = 0; t < 2; ++t) {
            const int dir = t ? 1 : -1;
            const int slot = irr ? rec[2 * d + t] : make_slot(SLOT_REG, 0, 0);
            const int type = slot_type(slot), j0 = slot_j(slot);
            for (int jj = 1; jj <= W; ++jj) {
                const int cd = ijk[d] + dir * jj;  // the neighbour's coordinate, then its image in the cell
                int64_t q = l + (int64_t)(dir * jj) * st[d];
                if (cd < 0) q += (int64_t)n * st[d];
                else if (cd >= n) q -= (int64_t)n * st[d];
                double val;
                if (type == SLOT_REG || jj < j0 || (labels[q] & KIND_MASK) == kind)
                    val = x[q];
                else
                    val = ghost[(int64_t)slot_cs(slot) * W + (jj - j0)];
                acc += ho_a<W>(jj) * val;
            }
        }
    return ((kind == K_PLUS) ? bp : bm) * inv_h2 * acc;
}

template <int DIM>
__global__ void __launch_bounds__(256) k_ho_apply_periodic(Box b, int n, const uint8_t* __restrict__ labels,
                                                           const int32_t* __restrict__ irr_index,
                                                           const int32_t* __restrict__ slots,
                                                           const double* __restrict__ ghost, double inv_h2, double bp,
                                                           double bm, const double* __restrict__ x,
                                                           double* __restrict__ y) {
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= b.size()) return;
    const uint8_t lab = labels[l];
    const uint8_t kind = lab & KIND_MASK;
    if (kind != K_PLUS && kind != K_MINUS) {
        y[l] = 0.0;
        return;
    }
    y[l] = ho_periodic_node<DIM>(b, n, l, lab, irr_index, slots, labels, ghost, inv_h2, bp, bm, x);
}

// the irregular nodes of a periodic cell, one thread each, from their list
template <int DIM>
__global__ void __launch_bounds__(256) k_ho_irregular_periodic(Box b, int n, const int32_t* __restrict__ nodes,
                                                               int64_t nirr, const uint8_t* __restrict__ labels,
                                                               const int32_t* __restrict__ irr_index,
                                                               const int32_t* __restrict__ slots,
                                                               const double* __restrict__ ghost, double inv_h2,
                                                               double bp, double bm, const double* __restrict__ x,
                                                               double* __restrict__ y) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nirr) return;
    const int64_t l = nodes[t];
    y[l] = ho_periodic_node<DIM>(b, n, l, labels[l], irr_index, slots, labels, ghost, inv_h2, bp, bm, x);
}


// Block index -> tile index such that each XCD (blocks are dealt to the 8 XCDs
// round robin) receives one contiguous run of tiles: neighbouring tiles then
// share that XCD's L2.
__device__ inline int xcd_tile(int bid, int nb) {
    const int xcd = bid & 7, idx = bid >> 3, per = nb >> 3, rem = nb & 7;
    return xcd * per + min(xcd, rem) + idx;
}

// (x, y, z) block coordinates of a one-dimensional launch of gx * gy * gz
// blocks, taken in XCD-contiguous order (x fastest)
struct Blk3 {
    int x, y, z;
};
__device__ inline Blk3 xcd_block3(int gx, int gy) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    return {t % gx, (t / gx) % gy, t / (gx * gy)};
}

// 3D apply of the regular unknowns, marching along z, for stencil half-width
// W (2: the (4,5) scheme, 3: the (6,7) scheme).  A block of 64 x 4 threads
// owns a 64 x (4 ZM_RY) tile of (x, y) columns (each thread ZM_RY rows) and a
// chunk of zc planes.  The z-neighbours of each column stay in a register
// queue (planes z - W .. z + W + 1); the x/y neighbours of the current plane
// come from an LDS copy of the tile with a W-node halo.  Every load is issued
// at least one plane ahead of its use (interior values one plane, halo values
// and labels W + 1), so the loads of a plane overlap the work on the previous
// ones.  One row per thread keeps the kernel at about 60 registers, eight
// waves per SIMD at W = 2 (six at W = 3, whose longer queue would spill at
// eight): twice the loads in flight of four rows at four waves (the march is
// bound by the loads it has in flight).  Irregular nodes are left to
// k_ho_irregular.
constexpr int ZM_TX = 64, ZM_RY = 1, ZM_TY = 4 * ZM_RY;

// PER: a periodic cell (the box itself, dims n, no margin): every load takes the
// image of its node in the cell.
template <int W, bool PER = false>
__global__ void __launch_bounds__(256, W == 2 ? 8 : 6) k_ho_apply3_zm(Box b, int3 clo, int3 chi, int ntx, int nty, int zc,
                                                      const uint8_t* __restrict__ labels, double inv_h2, double bp,
                                                      double bm, const double* __restrict__ x,
                                                      double* __restrict__ y) {
    constexpr int LA = W + 1;             // lookahead of the halo and label loads (planes)
    constexpr int NQ = 2 * W + 2;         // z queue: planes z - W .. z + W + 1
    constexpr int NHY = (2 * W + 3) / 4;  // y-halo rows per wavefront
    __shared__ double tile[ZM_TY + 2 * W][ZM_TX + 2 * W];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    const int i0 = clo.x + tx * ZM_TX, j0 = clo.y + ty * ZM_TY;
    const int i = i0 + lane;
    const int zs = clo.z + tz * zc, ze = min(zs + zc - 1, chi.z);
    const int bxh = b.lo[0] + b.dims[0] - 1, byh = b.lo[1] + b.dims[1] - 1, bzh = b.lo[2] + b.dims[2] - 1;
    const int n = b.dims[0];
    // in-box loads (the box holds the core with a W-node margin; beyond it in x/y: 0);
    // periodic: the column index is wrapped once per thread, rows and planes per load
    auto ldx = [&](int ii, int jj, int kk) -> double {
        if constexpr (PER) return x[b.idx(ii, wrap_near(jj, n), wrap_near(kk, n))];
        return (ii <= bxh && jj <= byh) ? x[b.idx(ii, jj, kk)] : 0.0;
    };
    const int iw = PER ? wrap_index(i, n) : i;
    auto ldl = [&](int jj, int kk) -> int {
        if constexpr (PER) return (int)labels[b.idx(iw, wrap_near(jj, n), wrap_near(kk, n))];
        return (i <= bxh && jj <= byh) ? (int)labels[b.idx(i, jj, kk)] : 0;
    };
    // x-halo duty: lanes 0 .. 2W-1 load tile columns 0 .. W-1 and ZM_TX+W .. ZM_TX+2W-1
    // of the thread's rows; y-halo duty: halo row k (rows 0 .. W-1, then
    // ZM_TY+W .. ZM_TY+2W-1) is loaded by wavefront k % 4, as its slot k / 4
    const int hcol = lane < W ? lane : ZM_TX + lane;
    const int hi = PER ? wrap_index(i0 - W + hcol, n) : i0 - W + hcol;
    int hr[NHY], hj[NHY];
#pragma unroll
    for (int u = 0; u < NHY; ++u) {
        const int k = wy + 4 * u;
        hr[u] = k < 2 * W ? (k < W ? k : ZM_TY + k) : -1;
        hj[u] = j0 - W + hr[u];
    }
    double q[ZM_RY][NQ];
    double hx[LA][ZM_RY], hy[LA][NHY];  // planes z .. z + W
    uint32_t lb[LA];                    // labels of the ZM_RY rows, one byte each
#pragma unroll
    for (int r = 0; r < ZM_RY; ++r)
#pragma unroll
        for (int d = 0; d < NQ - 1; ++d) q[r][d] = ldx(iw, j0 + wy + 4 * r, zs - W + d);
#pragma unroll
    for (int s = 0; s < LA; ++s) {
        const int zz = PER ? zs + s : min(zs + s, bzh);
        lb[s] = 0;
#pragma unroll
        for (int r = 0; r < ZM_RY; ++r) {
            hx[s][r] = lane < 2 * W ? ldx(hi, j0 + wy + 4 * r, zz) : 0.0;
            lb[s] |= (uint32_t)ldl(j0 + wy + 4 * r, zz) << (8 * r);
        }
#pragma unroll
        for (int u = 0; u < NHY; ++u) hy[s][u] = hr[u] >= 0 ? ldx(iw, hj[u], zz) : 0.0;
    }
    for (int z = zs; z <= ze; ++z) {
        const int zp = PER ? z + LA : min(z + LA, bzh);  // clamped planes are never used
        double hxn[ZM_RY], hyn[NHY];
        uint32_t lbn = 0;
#pragma unroll
        for (int r = 0; r < ZM_RY; ++r) {
            q[r][NQ - 1] = ldx(iw, j0 + wy + 4 * r, zp);
            hxn[r] = lane < 2 * W ? ldx(hi, j0 + wy + 4 * r, zp) : 0.0;
            lbn |= (uint32_t)ldl(j0 + wy + 4 * r, zp) << (8 * r);
        }
#pragma unroll
        for (int u = 0; u < NHY; ++u) hyn[u] = hr[u] >= 0 ? ldx(iw, hj[u], zp) : 0.0;
#pragma unroll
        for (int r = 0; r < ZM_RY; ++r) {
            tile[wy + 4 * r + W][lane + W] = q[r][W];
            if (lane < 2 * W) tile[wy + 4 * r + W][hcol] = hx[0][r];
        }
#pragma unroll
        for (int u = 0; u < NHY; ++u)
            if (hr[u] >= 0) tile[hr[u]][lane + W] = hy[0][u];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ZM_RY; ++r) {
            const int j = j0 + wy + 4 * r;
            const uint8_t lab = (uint8_t)(lb[0] >> (8 * r));
            const uint8_t kind = lab & KIND_MASK;
            if (i <= chi.x && j <= chi.y && !(lab & F_HO_IRR)) {
                const int64_t l = b.idx(i, j, z);
                if (kind != K_PLUS && kind != K_MINUS) {
                    y[l] = 0.0;
                } else {
                    const int tr = wy + 4 * r + W, tc = lane + W;
                    double acc;
                    if constexpr (W == 2) {
                        acc = 3.0 * A0 * q[r][2];
                        acc += A1 * (tile[tr][tc + 1] + tile[tr][tc - 1]) + A2 * (tile[tr][tc + 2] + tile[tr][tc - 2]);
                        acc += A1 * (tile[tr + 1][tc] + tile[tr - 1][tc]) + A2 * (tile[tr + 2][tc] + tile[tr - 2][tc]);
                        acc += A1 * (q[r][3] + q[r][1]) + A2 * (q[r][4] + q[r][0]);
                    } else {
                        acc = 3.0 * ho_a<W>(0) * q[r][W];
#pragma unroll
                        for (int jj = 1; jj <= W; ++jj)
                            acc += ho_a<W>(jj) * ((tile[tr][tc + jj] + tile[tr][tc - jj]) +
                                                  (tile[tr + jj][tc] + tile[tr - jj][tc]) + (q[r][W + jj] + q[r][W - jj]));
                    }
                    y[l] = ((kind == K_PLUS) ? bp : bm) * inv_h2 * acc;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ZM_RY; ++r) {
#pragma unroll
            for (int d = 0; d < NQ - 1; ++d) q[r][d] = q[r][d + 1];
#pragma unroll
            for (int s = 0; s < LA - 1; ++s) hx[s][r] = hx[s + 1][r];
            hx[LA - 1][r] = hxn[r];
        }
#pragma unroll
        for (int s = 0; s < LA - 1; ++s) {
#pragma unroll
            for (int u = 0; u < NHY; ++u) hy[s][u] = hy[s + 1][u];
            lb[s] = lb[s + 1];
        }
#pragma unroll
        for (int u = 0; u < NHY; ++u) hy[LA - 1][u] = hyn[u];
        lb[LA - 1] = lbn;
    }
}

// irregular nodes of the high-order apply, one thread each, from their list
template <int DIM, int W>
__global__ void __launch_bounds__(256) k_ho_irregular(Box b, const int32_t* __restrict__ nodes, int64_t nirr,
                                                      const uint8_t* __restrict__ labels,
                                                      const int32_t* __restrict__ irr_index,
                                                      const int32_t* __restrict__ slots,
                                                      const double* __restrict__ ghost,
                                                      const double* __restrict__ boxval, int w, double inv_h2,
                                                      double bp, double bm, const double* __restrict__ x,
                                                      double* __restrict__ y, int with_data) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nirr) return;
    const int64_t l = nodes[t];
    const uint8_t kind = labels[l] & KIND_MASK;
    double acc = (double)DIM * ho_a<W>(0) * x[l];
    acc += ho_irregular<DIM, W>(b, l, kind, labels, slots + (int64_t)irr_index[l] * 2 * DIM, ghost, boxval, x,
                                with_data);
    y[l] = ((kind == K_PLUS) ? bp : bm) * inv_h2 * acc;
}

void run_ho_apply_periodic(int dim, const Box& b, int n, const uint8_t* labels, const int32_t* irr_index,
                           const int32_t* slots, const int32_t* irr_nodes, int64_t nirr, const double* ghost,
                           double inv_h2, double beta_plus, double beta_minus, const double* x, double* y,
                           hipStream_t s, int part) {
    const int64_t N = b.size();
    if (N == 0) return;
    if (dim == 2) {
        hipLaunchKernelGGL((k_ho_apply_periodic<2>), dim3(cdiv(N, 256)), dim3(256), 0, s, b, n, labels, irr_index,
                           slots, ghost, inv_h2, beta_plus, beta_minus, x, y);
        IIM_LAUNCH_CHECK();
        return;
    }
    // 3D: the z-march over the cell (loads wrapped), then the irregular nodes from their list
    for (int d = 0; d < 3; ++d)
        if (b.lo[d] != 0 || b.dims[d] != n) throw Error(IIM_E_INTERNAL, "apply: the periodic box must be the cell");
    const int3 lo = make_int3(0, 0, 0), hi = make_int3(n - 1, n - 1, n - 1);
    const int ntx = cdiv(n, ZM_TX), nty = cdiv(n, ZM_TY);
    const int64_t cols = (int64_t)ntx * nty;
    const int zc = (int)std::max<int64_t>(8, std::min<int64_t>(16, cols * n / 2048));
    const int64_t nb = cols * cdiv(n, zc);
    if (part != 2) {
        hipLaunchKernelGGL((k_ho_apply3_zm<2, true>), dim3((unsigned)nb), dim3(256), 0, s, b, lo, hi, ntx, nty, zc,
                           labels, inv_h2, beta_plus, beta_minus, x, y);
        IIM_LAUNCH_CHECK();
    }
    if (nirr > 0 && part != 1) {
        hipLaunchKernelGGL((k_ho_irregular_periodic<3>), dim3(cdiv(nirr, 256)), dim3(256), 0, s, b, n, irr_nodes, nirr,
                           labels, irr_index, slots, ghost, inv_h2, beta_plus, beta_minus, x, y);
        IIM_LAUNCH_CHECK();
    }
}

void run_ho_apply(int dim, const Box& b, const int* core_lo, const int* core_hi, const uint8_t* labels,
                  const int32_t* irr_index, const int32_t* slots, const int32_t* irr_nodes, int64_t nirr,
                  const double* ghost, const double* boxval, int w, double inv_h2, double beta_plus,
                  double beta_minus, const double* x, double* y, int with_data, hipStream_t s, int part) {
    int3 lo = make_int3(core_lo[0], core_lo[1], core_lo[2]);
    int3 hi = make_int3(core_hi[0], core_hi[1], core_hi[2]);
    int nx = hi.x - lo.x + 1, ny = hi.y - lo.y + 1, nz = hi.z - lo.z + 1;
    if (nx <= 0 || ny <= 0 || nz <= 0) return;
    if (dim == 3) {
        // the z-march reads planes zs-w .. ze+w and columns/rows up to w past the
        // core: the storage box has that margin
        if (w != 2 && w != 3) throw Error(IIM_E_INTERNAL, "apply: stencil half-width must be 2 or 3");
        for (int d = 0; d < 3; ++d)
            if (core_lo[d] - w < b.lo[d] || core_hi[d] + w > b.lo[d] + b.dims[d] - 1)
                throw Error(IIM_E_INTERNAL, "apply: storage box lacks the stencil margin");
        const int ntx = cdiv(nx, ZM_TX), nty = cdiv(ny, ZM_TY);
        const int64_t cols = (int64_t)ntx * nty;
        // chunks of 8..16 planes, shorter when the tiles are too few to fill the device
        int zc = (int)std::max<int64_t>(8, std::min<int64_t>(16, cols * nz / 2048));
        const int nzc = cdiv(nz, zc);
        const int64_t nb = cols * nzc;
        if (part != 2) {
            if (w == 2)
                hipLaunchKernelGGL((k_ho_apply3_zm<2>), dim3((unsigned)nb), dim3(256), 0, s, b, lo, hi, ntx, nty, zc,
                                   labels, inv_h2, beta_plus, beta_minus, x, y);
            else
                hipLaunchKernelGGL((k_ho_apply3_zm<3>), dim3((unsigned)nb), dim3(256), 0, s, b, lo, hi, ntx, nty, zc,
                                   labels, inv_h2, beta_plus, beta_minus, x, y);
            IIM_LAUNCH_CHECK();
        }
        if (nirr > 0 && part != 1) {
            if (w == 2)
                hipLaunchKernelGGL((k_ho_irregular<3, 2>), dim3(cdiv(nirr, 256)), dim3(256), 0, s, b, irr_nodes, nirr,
                                   labels, irr_index, slots, ghost, boxval, w, inv_h2, beta_plus, beta_minus, x, y,
                                   with_data);
            else
                hipLaunchKernelGGL((k_ho_irregular<3, 3>), dim3(cdiv(nirr, 256)), dim3(256), 0, s, b, irr_nodes, nirr,
                                   labels, irr_index, slots, ghost, boxval, w, inv_h2, beta_plus, beta_minus, x, y,
                                   with_data);
            IIM_LAUNCH_CHECK();
        }
        return;
    }
    if (part == 2) return;  // 2D: irregular nodes are inside the one stencil kernel
    dim3 blk(64, 4, 1);
    dim3 grd(cdiv(nx, 64), cdiv(ny, 4), 1);
    if (w == 2)
        hipLaunchKernelGGL((k_ho_apply<2, 2>), grd, blk, 0, s, b, lo, hi, labels, irr_index, slots, ghost, boxval,
                           inv_h2, beta_plus, beta_minus, x, y, with_data);
    else if (w == 3)
        hipLaunchKernelGGL((k_ho_apply<2, 3>), grd, blk, 0, s, b, lo, hi, labels, irr_index, slots, ghost, boxval,
                           inv_h2, beta_plus, beta_minus, x, y, with_data);
    else
        throw Error(IIM_E_INTERNAL, "apply: stencil half-width must be 2 or 3");
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// post-processing of a solution (Sec. 2.4 of the paper)
// ---------------------------------------------------------------------------
// grad u at the unknowns: per axis the central first derivative of order 2W
// over the extended function (the Laplacian's ghost values and box
// extrapolation), written to grad[d * total + full-grid index]; one thread per
// node of the core, nodes that are no unknowns are left alone.
template <int DIM, int W>
__global__ void __launch_bounds__(256) k_ho_gradient(Box b, int3 clo, int3 chi, int n, const uint8_t* __restrict__ labels,
                                                     const int32_t* __restrict__ irr_index,
                                                     const int32_t* __restrict__ slots, const double* __restrict__ ghost,
                                                     const double* __restrict__ boxval, double inv_h,
                                                     const double* __restrict__ x, double* __restrict__ grad,
                                                     int64_t total) {
    const int i = clo.x + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = clo.y + blockIdx.y * blockDim.y + threadIdx.y;
    const int k = DIM == 3 ? clo.z + (int)blockIdx.z : 0;
    if (i > chi.x || j > chi.y) return;
    if (i < 0 || i > n || j < 0 || j > n || k < 0 || k > n) return;
    const int64_t l = b.idx(i, j, k);
    const uint8_t lab = labels[l];
    const uint8_t kind = lab & KIND_MASK;
    if (kind != K_PLUS && kind != K_MINUS) return;
    const int64_t f = i + (int64_t)(n + 1) * (j + (int64_t)(n + 1) * k);
    const int64_t st[3] = {1, (int64_t)b.dims[0], (int64_t)b.dims[0] * b.dims[1]};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double vp[W], vm[W];
        if (lab & F_HO_IRR) {
            const int32_t* rec = slots + (int64_t)irr_index[l] * 2 * DIM;
            ho_half_line<W>(l, -st[d], rec[2 * d + 0], kind, labels, ghost, boxval, x, 1, vm);
            ho_half_line<W>(l, st[d], rec[2 * d + 1], kind, labels, ghost, boxval, x, 1, vp);
        } else {
#pragma unroll
            for (int jj = 1; jj <= W; ++jj) {
                vp[jj - 1] = x[l + jj * st[d]];
                vm[jj - 1] = x[l - jj * st[d]];
            }
        }
        double g = 0.0;
#pragma unroll
        for (int jj = 1; jj <= W; ++jj) g += ho_g<W>(jj) * (vp[jj - 1] - vm[jj - 1]);
        grad[(int64_t)d * total + f] = g * inv_h;
    }
}

void run_ho_gradient(int dim, const Box& b, const int* core_lo, const int* core_hi, int n, const uint8_t* labels,
                     const int32_t* irr_index, const int32_t* slots, const double* ghost, const double* boxval, int w,
                     double inv_h, const double* x, double* grad, hipStream_t s) {
    const int3 lo = make_int3(core_lo[0], core_lo[1], core_lo[2]);
    const int3 hi = make_int3(core_hi[0], core_hi[1], core_hi[2]);
    const int nx = hi.x - lo.x + 1, ny = hi.y - lo.y + 1, nz = dim == 3 ? hi.z - lo.z + 1 : 1;
    if (nx <= 0 || ny <= 0 || nz <= 0) return;
    // every stencil point of a core node lies in the storage box (w-node margin)
    for (int d = 0; d < dim; ++d)
        if (core_lo[d] - w < b.lo[d] || core_hi[d] + w > b.lo[d] + b.dims[d] - 1)
            throw Error(IIM_E_INTERNAL, "gradient: storage box lacks the stencil margin");
    const int64_t total = dim == 2 ? (int64_t)(n + 1) * (n + 1) : (int64_t)(n + 1) * (n + 1) * (n + 1);
    const dim3 blk(64, 4, 1);
    const dim3 grd(cdiv(nx, 64), cdiv(ny, 4), nz);
    if (dim == 3 && w == 2)
        hipLaunchKernelGGL((k_ho_gradient<3, 2>), grd, blk, 0, s, b, lo, hi, n, labels, irr_index, slots, ghost,
                           boxval, inv_h, x, grad, total);
    else if (dim == 3 && w == 3)
        hipLaunchKernelGGL((k_ho_gradient<3, 3>), grd, blk, 0, s, b, lo, hi, n, labels, irr_index, slots, ghost,
                           boxval, inv_h, x, grad, total);
    else if (dim == 2 && w == 2)
        hipLaunchKernelGGL((k_ho_gradient<2, 2>), grd, blk, 0, s, b, lo, hi, n, labels, irr_index, slots, ghost,
                           boxval, inv_h, x, grad, total);
    else if (dim == 2 && w == 3)
        hipLaunchKernelGGL((k_ho_gradient<2, 3>), grd, blk, 0, s, b, lo, hi, n, labels, irr_index, slots, ghost,
                           boxval, inv_h, x, grad, total);
    else
        throw Error(IIM_E_INTERNAL, "gradient: unsupported dimension / half-width");
    IIM_LAUNCH_CHECK();
}

// The boundary quantity the condition leaves open, one value per control
// point: with s the fit's normal-derivative row (row w of S, its u(x_c)
// weight s_c) and dot = sum_i s_i u_i over the fit's nodes,
//   Dirichlet  du/dn(x_c) = s_c ubar + dot;
//   Neumann    u(x_c) = (qbar - beta+ dot) / (beta+ s_c);
//   interface  du+/dn(x_c) = s+_c u+(x_c) + dot+, u+(x_c) from the closure
//              (D = beta+ s+_c - beta- s-_c).
// GLN lanes per control point gather the dot products.
template <int NS, int GLN>
__global__ void __launch_bounds__(256) k_boundary_quantity(BQDev B, const double* __restrict__ x,
                                                           const double* __restrict__ cpdata, double* __restrict__ q) {
    const int lane = threadIdx.x % GLN;
    const int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / GLN;
    if (c >= B.ncp) return;  // whole groups exit together
    double dots[NS];
#pragma unroll
    for (int sd = 0; sd < NS; ++sd) {
        const int64_t cs = c * NS + sd;
        double acc = 0.0;
        for (int64_t a = B.ptr[cs] + lane; a < B.ptr[cs + 1]; a += GLN) acc += B.Sd[a] * x[B.idx[a]];
#pragma unroll
        for (int off = GLN / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, GLN);
        dots[sd] = acc;
    }
    if (lane != 0) return;
    const int nr = B.nrows, w = B.w;
    const double bp = B.beta_plus;
    if (NS == 1) {
        const double scn = B.Sc[c * nr + w];
        q[c] = B.bc == IIM_BC_DIRICHLET ? scn * cpdata[c] + dots[0] : (cpdata[c] - bp * dots[0]) / (bp * scn);
        return;
    }
    const double bm = B.beta_minus;
    const double scp = B.Sc[(c * 2 + 0) * nr + w], scm = B.Sc[(c * 2 + 1) * nr + w];
    const double D = bp * scp - bm * scm;
    const double ubar = -(bp * dots[0] - bm * dots[NS - 1]) / D;
    const double up = ubar + (cpdata[2 * c + 1] - bm * scm * cpdata[2 * c]) / D;
    q[c] = scp * up + dots[0];
}

void run_boundary_quantity(const BQDev& B, const double* x, const double* cpdata, double* q, hipStream_t s) {
    if (B.ncp == 0) return;
    if (B.nrows != B.w + 1) throw Error(IIM_E_INTERNAL, "boundary quantity: the fits lack the derivative row");
    const int64_t threads = B.ncp * 64;
    if (B.nsides == 1)
        hipLaunchKernelGGL((k_boundary_quantity<1, 64>), dim3(cdiv(threads, 256)), dim3(256), 0, s, B, x, cpdata, q);
    else
        hipLaunchKernelGGL((k_boundary_quantity<2, 64>), dim3(cdiv(threads, 256)), dim3(256), 0, s, B, x, cpdata, q);
    IIM_LAUNCH_CHECK();
}

// One wave per control point, lanes over the fit's entries (coalesced rows):
// the dot products of rows d/dn and d/dx_d with the solution, then on lane 0
// the fit's value at x_c (Dirichlet: ubar; Neumann: the closure of the normal
// row; interface: u+(x_c) from the interface closure, as the boundary
// quantity), and grad_d = s^d_c U_c + sum_i s^d_i u_i.  With cp, also the
// pressure coefficient of the wall velocity grad + U.
template <int NS, int DIM>
__global__ void __launch_bounds__(256) k_wall_gradient(WGDev G, const double* __restrict__ x,
                                                       const double* __restrict__ cpdata, double* __restrict__ grad,
                                                       double* __restrict__ cp) {
    constexpr int GLN = 64, NR = 1 + DIM;
    const int lane = threadIdx.x % GLN;
    const int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / GLN;
    if (c >= G.ncp) return;  // whole waves exit together
    int64_t nnz = G.ptr[G.ncp * NS];
    double dot[NR], dotm = 0.0;
    {
        const int64_t cs = c * NS;
#pragma unroll
        for (int r = 0; r < NR; ++r) dot[r] = 0.0;
        for (int64_t a = G.ptr[cs] + lane; a < G.ptr[cs + 1]; a += GLN) {
            const double xv = x[G.idx[a]];
#pragma unroll
            for (int r = 0; r < NR; ++r) dot[r] += G.S[r * nnz + a] * xv;
        }
#pragma unroll
        for (int r = 0; r < NR; ++r)
            for (int off = GLN / 2; off > 0; off >>= 1) dot[r] += __shfl_xor(dot[r], off, GLN);
        if (NS == 2) {
            for (int64_t a = G.ptr[cs + 1] + lane; a < G.ptr[cs + 2]; a += GLN) dotm += G.S[a] * x[G.idx[a]];
            for (int off = GLN / 2; off > 0; off >>= 1) dotm += __shfl_xor(dotm, off, GLN);
        }
    }
    if (lane != 0) return;
    const double bp = G.beta_plus;
    const double* scp = G.Sc + (c * NS) * NR;
    double uc;
    if (NS == 1) {
        uc = G.bc == IIM_BC_DIRICHLET ? cpdata[c] : (cpdata[c] - bp * dot[0]) / (bp * scp[0]);
    } else {
        const double bm = G.beta_minus;
        const double scm = G.Sc[(c * 2 + 1) * NR];
        const double D = bp * scp[0] - bm * scm;
        const double ubar = -(bp * dot[0] - bm * dotm) / D;
        uc = ubar + (cpdata[2 * c + 1] - bm * scm * cpdata[2 * c]) / D;
    }
    double v2 = 0.0, u2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double g = scp[1 + d] * uc + dot[1 + d];
        grad[c * DIM + d] = g;
        const double vd = g + G.u_inf[d];
        v2 += vd * vd;
        u2 += G.u_inf[d] * G.u_inf[d];
    }
    if (cp) cp[c] = 1.0 - v2 / u2;
}

void run_wall_gradient(const WGDev& G, const double* x, const double* cpdata, double* grad, double* cp,
                       hipStream_t s) {
    if (G.ncp == 0) return;
    const int64_t threads = G.ncp * 64;
    const dim3 grid(cdiv(threads, 256)), blk(256);
    if (G.dim == 2) {
        if (G.nsides == 1) hipLaunchKernelGGL((k_wall_gradient<1, 2>), grid, blk, 0, s, G, x, cpdata, grad, cp);
        else hipLaunchKernelGGL((k_wall_gradient<2, 2>), grid, blk, 0, s, G, x, cpdata, grad, cp);
    } else {
        if (G.nsides == 1) hipLaunchKernelGGL((k_wall_gradient<1, 3>), grid, blk, 0, s, G, x, cpdata, grad, cp);
        else hipLaunchKernelGGL((k_wall_gradient<2, 3>), grid, blk, 0, s, G, x, cpdata, grad, cp);
    }
    IIM_LAUNCH_CHECK();
}

__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void run_fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 4096)), dim3(256), 0, s, p, n, v);
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Shortley-Weller level kernels (scaled rows: h^2 x operator)
// ---------------------------------------------------------------------------
template <typename T> __device__ inline const T* rec_ptr(const LevelDev& L);
template <> __device__ inline const float* rec_ptr<float>(const LevelDev& L) { return L.rec32; }
template <> __device__ inline const double* rec_ptr<double>(const LevelDev& L) { return L.rec64; }

__device__ inline float to_f(float v) { return v; }
__device__ inline float to_f(__half v) { return __half2float(v); }
__device__ inline __half from_f(float v, __half*) { return __float2half(v); }
__device__ inline float from_f(float v, float*) { return v; }

// load an iterate of storage type S as arithmetic type T
template <typename T, typename S> __device__ inline T load_it(const S* p, int64_t i) { return (T)to_f(p[i]); }
template <> __device__ inline double load_it<double, double>(const double* p, int64_t i) { return p[i]; }

// store a value of arithmetic type T into storage type S
template <typename T, typename S> __device__ inline void store_t(S* p, int64_t i, T v) {
    p[i] = from_f((float)v, (S*)nullptr);
}
template <> __device__ inline void store_t<double, double>(double* p, int64_t i, double v) { p[i] = v; }
// v rounded to the storage type S (kept in T)
template <typename T, typename S>
__device__ inline T round_s(T v) { return (T)to_f(from_f((float)v, (S*)nullptr)); }
template <> __device__ inline double round_s<double, double>(double v) { return v; }

// Shortley-Weller row at an unknown from its neighbour values: diagonal and
// off-diagonal sum (zm[d], zp[d] = z at the neighbours (d, -) and (d, +))
template <typename T, int DIM>
__device__ inline void sw_combine(const LevelDev& L, int64_t l, uint8_t lab, const T* zm, const T* zp, T* diag,
                                  T* off) {
    T acc = 0;
    if (!(lab & F_SW_IRR)) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) acc += zp[d] + zm[d];
        *diag = (T)(-2 * DIM);
    } else {
        const T* rec = rec_ptr<T>(L) + (int64_t)L.irr_index[l] * (1 + 2 * DIM);
#pragma unroll
        for (int d = 0; d < DIM; ++d) acc += rec[1 + 2 * d] * zm[d] + rec[2 + 2 * d] * zp[d];
        *diag = rec[0];
    }
    *off = acc;
}

// (A' z) and the diagonal at the unknown (i, j, k) (box index l, label lab);
// off-diagonal sum returned in *off.  Neighbour z in the level's layout.
template <typename T, typename S, int DIM>
__device__ inline void sw_row(const LevelDev& L, int i, int j, int k, int64_t l, uint8_t lab, const S* z, T* diag,
                              T* off) {
    int64_t nm[3], np[3];  // indices of the neighbours (d, -) and (d, +)
    if (!L.split) {
        const int64_t st[3] = {1, (int64_t)L.box.dims[0], (int64_t)L.box.dims[0] * L.box.dims[1]};
        const int c[3] = {i, j, k};
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            nm[d] = l - st[d];
            np[d] = l + st[d];
            if (L.periodic) {  // the box is the periodic cell
                if (c[d] == 0) nm[d] = l + (int64_t)(L.n - 1) * st[d];
                if (c[d] == L.n - 1) np[d] = l - (int64_t)(L.n - 1) * st[d];
            }
        }
    } else {
        // neighbours have the other colour: rows r, r +- 1, r +- dims_y of that array
        const int a = i - L.box.lo[0];
        const int64_t r = (int64_t)(j - L.box.lo[1]) + (int64_t)L.box.dims[1] * (k - L.box.lo[2]);
        const int64_t base = (int64_t)(((i + j + k) & 1) ^ 1) * L.half + r * L.hx;
        const int64_t ry = L.hx, rz = (int64_t)L.hx * L.box.dims[1];
        nm[0] = base + ((a - 1) >> 1);
        np[0] = base + ((a + 1) >> 1);
        nm[1] = base - ry + (a >> 1);
        np[1] = base + ry + (a >> 1);
        nm[2] = base - rz + (a >> 1);
        np[2] = base + rz + (a >> 1);
        if (L.periodic) {  // the box is the cell (lo 0, n per axis): neighbours across the seam
            const int n = L.n;
            if (i == 0) nm[0] = base + ((n - 1) >> 1);
            if (i == n - 1) np[0] = base;
            if (j == 0) nm[1] = base + (int64_t)(n - 1) * ry + (a >> 1);
            if (j == n - 1) np[1] = base - (int64_t)(n - 1) * ry + (a >> 1);
            if (k == 0) nm[2] = base + (int64_t)(n - 1) * rz + (a >> 1);
            if (k == n - 1) np[2] = base - (int64_t)(n - 1) * rz + (a >> 1);
        }
    }
    T zm[3], zp[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        zm[d] = load_it<T, S>(z, nm[d]);
        zp[d] = load_it<T, S>(z, np[d]);
    }
    sw_combine<T, DIM>(L, l, lab, zm, zp, diag, off);
}

// ---- per-node bodies shared by the grid kernels and the single-workgroup tail
template <typename T, typename S, int DIM>
__device__ inline void rbgs_node(const LevelDev& L, int i, int j, int k, int colour, S* z, const T* b) {
    if (((i + j + k) & 1) != colour) return;
    const int64_t l = L.box.idx(i, j, k);
    const uint8_t lab = L.labels[l];
    if (!is_unknown(lab)) return;
    T diag, off;
    sw_row<T, S, DIM>(L, i, j, k, l, lab, z, &diag, &off);
    const int64_t v = vidx(L, i, j, k);
    if (diag != (T)0) store_t<T, S>(z, v, (b[v] - off) / diag);
}

// residual of the fine level at an in-box node (zero off the unknowns)
template <typename T, typename S, int DIM>
__device__ inline T fine_resid(const LevelDev& F, int i, int j, int k, const S* z, const T* b) {
    const int64_t l = F.box.idx(i, j, k);
    const uint8_t lab = F.labels[l];
    if (!is_unknown(lab)) return (T)0;
    T diag, off;
    sw_row<T, S, DIM>(F, i, j, k, l, lab, z, &diag, &off);
    const int64_t v = vidx(F, i, j, k);
    return b[v] - (diag * load_it<T, S>(z, v) + off);
}

// coarse rhs (scaled by h_c^2 = 4 h_f^2): 4 * half-weighting of the fine residual
template <typename T, typename S, int DIM>
__device__ inline void restrict_node(const LevelDev& F, const LevelDev& C, int I, int J, int K, const S* z,
                                     const T* b, T* bc) {
    const int64_t lc = C.box.idx(I, J, K), vc = vidx(C, I, J, K);
    if (!is_unknown(C.labels[lc])) {
        bc[vc] = (T)0;
        return;
    }
    const int f2[3] = {2 * I, 2 * J, 2 * K};
    if (!F.periodic)
        for (int d = 0; d < DIM; ++d)
            if (f2[d] - 1 < F.box.lo[d] || f2[d] + 1 >= F.box.lo[d] + F.box.dims[d]) {
                bc[vc] = (T)0;  // cannot happen: a coarse unknown is a fine unknown
                return;
            }
    const T w0 = (T)0.5, w1 = DIM == 2 ? (T)0.125 : (T)(1.0 / 12.0);
    T acc = w0 * fine_resid<T, S, DIM>(F, f2[0], f2[1], f2[2], z, b);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        int p[3] = {f2[0], f2[1], f2[2]}, m[3] = {f2[0], f2[1], f2[2]};
        p[d] += 1;
        m[d] -= 1;
        if (F.periodic) {  // fine neighbours modulo n
            p[d] = wrap_near(p[d], F.n);
            m[d] = wrap_near(m[d], F.n);
        }
        acc += w1 * (fine_resid<T, S, DIM>(F, p[0], p[1], p[2], z, b) + fine_resid<T, S, DIM>(F, m[0], m[1], m[2], z, b));
    }
    bc[vc] = (T)4 * acc;
}

// (P z_c)(i, j, k) at a fine unknown; mode 0 = (bi/tri)linear, 1 = average of
// in-domain parents.  Returns false when no parent contributes.
template <typename T, typename S, int DIM>
__device__ inline bool prolong_corr(const LevelDev& C, int i, int j, int k, int mode, const S* zc, T* corr) {
    // parents: floor(f/2) and, along axes where f is odd, floor(f/2) + 1
    const int li = i >> 1, lj = j >> 1, lk = k >> 1;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (DIM == 3 && (k & 1)) ? 2 : 1;
    T sum = 0;
    int cnt = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bq = 0; bq < 2; ++bq)
#pragma unroll
            for (int cq = 0; cq < (DIM == 3 ? 2 : 1); ++cq) {
                if (a >= ni || bq >= nj || cq >= nk) continue;
                int P0 = li + a, P1 = lj + bq, P2 = lk + cq;
                if (C.periodic) {  // coarse parent n_c is the image of 0
                    P0 = wrap_near(P0, C.n);
                    P1 = wrap_near(P1, C.n);
                    if (DIM == 3) P2 = wrap_near(P2, C.n);
                }
                const bool inb = P0 >= C.box.lo[0] && P0 < C.box.lo[0] + C.box.dims[0] && P1 >= C.box.lo[1] &&
                                 P1 < C.box.lo[1] + C.box.dims[1] && P2 >= C.box.lo[2] &&
                                 P2 < C.box.lo[2] + C.box.dims[2];
                T v = 0;
                bool use = mode == 0;
                if (inb) {
                    const int64_t lp = C.box.idx(P0, P1, P2);
                    v = load_it<T, S>(zc, vidx(C, P0, P1, P2));
                    if (mode == 1) {
                        const uint8_t kk = C.labels[lp] & KIND_MASK;
                        use = kk == K_PLUS || kk == K_MINUS || kk == K_BOX;
                    }
                } else if (mode == 1) {
                    use = false;
                }
                if (use) {
                    sum += v;
                    cnt += 1;
                }
            }
    if (cnt == 0) return false;
    *corr = sum / (T)cnt;
    return true;
}

// z_f += P z_c at a fine unknown
template <typename T, typename S, int DIM>
__device__ inline void prolong_node(const LevelDev& F, const LevelDev& C, int i, int j, int k, int mode, const S* zc,
                                    S* z) {
    const int64_t l = F.box.idx(i, j, k);
    if (!is_unknown(F.labels[l])) return;
    T corr;
    const int64_t v = vidx(F, i, j, k);
    if (prolong_corr<T, S, DIM>(C, i, j, k, mode, zc, &corr)) store_t<T, S>(z, v, load_it<T, S>(z, v) + corr);
}

template <typename T, typename S>
__device__ inline void coarse_row(const int32_t* list, int64_t nc, const T* Ainv, const T* b, S* z, int64_t r) {
    T acc = 0;
    for (int64_t c = 0; c < nc; ++c) acc += Ainv[r * nc + c] * b[list[c]];
    store_t<T, S>(z, list[r], acc);
}

// ---- grid kernels
template <typename T, typename S, int DIM>
__global__ void __launch_bounds__(256) k_rbgs(LevelDev L, int colour, S* z, const T* b) {
    // one thread per pair of x-neighbours: the one of the colour being updated
    const int j = L.core_lo[1] + blockIdx.y * blockDim.y + threadIdx.y;
    const int k = DIM == 3 ? L.core_lo[2] + blockIdx.z : 0;
    const int i0 = L.core_lo[0] + 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int i = i0 + ((i0 + j + k + colour) & 1);
    if (i > L.core_hi[0] || j > L.core_hi[1]) return;
    rbgs_node<T, S, DIM>(L, i, j, k, colour, z, b);
}

template <typename T, typename S, int DIM>
__global__ void __launch_bounds__(256) k_sw_apply(LevelDev L, const S* z, T* y) {
    int i = L.core_lo[0] + blockIdx.x * blockDim.x + threadIdx.x;
    int j = L.core_lo[1] + blockIdx.y * blockDim.y + threadIdx.y;
    int k = DIM == 3 ? L.core_lo[2] + blockIdx.z : 0;
    if (i > L.core_hi[0] || j > L.core_hi[1]) return;
    const int64_t l = L.box.idx(i, j, k), v = vidx(L, i, j, k);
    const uint8_t lab = L.labels[l];
    if (!is_unknown(lab)) {
        y[v] = (T)0;
        return;
    }
    T diag, off;
    sw_row<T, S, DIM>(L, i, j, k, l, lab, z, &diag, &off);
    y[v] = diag * load_it<T, S>(z, v) + off;
}

// levels with at least this many entries per colour take four entries per thread
// in their half-sweeps (enough threads remain to fill the device)
constexpr int64_t SPLIT4_MIN_ENTRIES = 1 << 20;

// four consecutive entries of a level vector (16-byte aligned: the entry index is
// a multiple of 4 and rows hold a multiple of 4 entries), converted to T
template <typename S>
struct alignas(4 * sizeof(S)) Vec4 {
    S v[4];
};
template <typename T, typename S>
__device__ inline void ld4(const S* p, int e, T (&out)[4]) {
    const Vec4<S> q = *reinterpret_cast<const Vec4<S>*>(p + e);
#pragma unroll
    for (int u = 0; u < 4; ++u) out[u] = load_it<T, S>(q.v, u);
}

// Half-sweep on a colour-split 3D level.  A thread owns four consecutive
// entries m0..m0+3 of its colour in one box row (nodes x = lo + 2m + parity of
// the row) and loads, as 16-byte vectors, their labels, right-hand sides and
// the other colour's entries in the rows beside them (y +- 1, z +- 1) and in
// their own row (plus one entry at either end for the x-neighbours).  Every load
// is issued before the first test (the neighbours of core rows lie in the box).
// Threads run over (core row, quad) pairs without gaps (nq = hx / 4 quads a
// row, ny core rows a plane, nrows core rows), blocks in XCD-contiguous order:
// a row of 49 quads (cfg-4 level 0) left 15 of 64 lanes idle.  Rows are
// contiguous in a colour array, so lanes still read consecutive entries.
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_rbgs_split(LevelDev L, int colour, int nq, int ny, int nrows, S* z,
                                                    const T* b) {
    const int f = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int row = f / nq;
    if (row >= nrows) return;
    const int m0 = 4 * (f - row * nq);
    const int j = L.core_lo[1] + row % ny;
    const int k = L.core_lo[2] + row / ny;
    const int p = (colour ^ (L.box.lo[0] + j + k)) & 1;  // node of entry m: x offset a = 2m + p
    const int r = (j - L.box.lo[1]) + L.box.dims[1] * (k - L.box.lo[2]);
    const int own = colour * (int)L.half + r * L.hx + m0;
    const int oth = (colour ^ 1) * (int)L.half + r * L.hx + m0;
    const int ry = L.hx, rz = L.hx * L.box.dims[1];
    const uint32_t lab4 = *reinterpret_cast<const uint32_t*>(L.lab_split + own);
    // neighbour rows and the entries before and after the thread's four; on a
    // periodic cell (rows of exactly n / 2 entries) they wrap across the seam
    int oym = oth - ry, oyp = oth + ry, ozm = oth - rz, ozp = oth + rz, ocm = oth - 1, ocp = oth + 4;
    if (L.periodic) {
        const int n = L.n;
        if (j == 0) oym = oth + (n - 1) * ry;
        if (j == n - 1) oyp = oth - (n - 1) * ry;
        if (k == 0) ozm = oth + (n - 1) * rz;
        if (k == n - 1) ozp = oth - (n - 1) * rz;
        if (m0 == 0) ocm = oth + L.hx - 1;
        if (m0 + 4 == L.hx) ocp = oth - m0;
    }
    T bv[4], c4[4], ym[4], yp[4], zmv[4], zpv[4];
    ld4<T, T>(b, own, bv);
    ld4<T, S>(z, oth, c4);
    ld4<T, S>(z, oym, ym);
    ld4<T, S>(z, oyp, yp);
    ld4<T, S>(z, ozm, zmv);
    ld4<T, S>(z, ozp, zpv);
    const T cm = load_it<T, S>(z, ocm), cp = load_it<T, S>(z, ocp);  // in the box: core rows
    asm volatile("" ::"v"(lab4), "v"(bv[0]), "v"(c4[0]), "v"(ym[0]), "v"(yp[0]), "v"(zmv[0]), "v"(zpv[0]), "v"(cm),
                 "v"(cp));
    T out[4];
    int done = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint8_t lab = (uint8_t)(lab4 >> (8 * u));
        const int a = 2 * (m0 + u) + p, i = L.box.lo[0] + a;
        out[u] = (T)0;
        if (i < L.core_lo[0] || i > L.core_hi[0] || !is_unknown(lab)) continue;
        T zm[3], zp[3];
        zm[0] = p ? c4[u] : (u == 0 ? cm : c4[u - 1]);  // entry (a - 1) >> 1
        zp[0] = p ? (u == 3 ? cp : c4[u + 1]) : c4[u];  // entry (a + 1) >> 1
        zm[1] = ym[u];
        zp[1] = yp[u];
        zm[2] = zmv[u];
        zp[2] = zpv[u];
        T diag, off;
        sw_combine<T, 3>(L, (int64_t)a + (int64_t)L.box.dims[0] * r, lab, zm, zp, &diag, &off);
        if (diag == (T)0) continue;
        out[u] = (bv[u] - off) / diag;
        done |= 1 << u;
    }
    if (done == 15) {
        Vec4<S> q;
#pragma unroll
        for (int u = 0; u < 4; ++u) store_t<T, S>(q.v, u, out[u]);
        *reinterpret_cast<Vec4<S>*>(z + own) = q;
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (done & (1 << u)) store_t<T, S>(z, own + u, out[u]);
    }
}

// Half-sweep on a colour-split 3D level, one entry per thread (levels too small
// to fill the device with four entries per thread): threads walk the colour's
// entries of each box row contiguously (x of the colour's nodes = lo_x + 2 m + offset).
// Every load is issued before the first use (the neighbours of a core node are
// in the box), and offsets are 32-bit (level vectors hold < 2^31 entries).
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_rbgs_split1(LevelDev L, int colour, int gx, int gy, S* z, const T* b) {
    const Blk3 B = xcd_block3(gx, gy);
    const int m = B.x * 64 + (threadIdx.x & 63);
    const int j = L.core_lo[1] + B.y * 4 + (threadIdx.x >> 6);
    const int k = L.core_lo[2] + B.z;
    if (j > L.core_hi[1] || m >= L.hx) return;
    const int i = L.box.lo[0] + 2 * m + ((colour ^ (L.box.lo[0] + j + k)) & 1);
    if (i < L.core_lo[0] || i > L.core_hi[0]) return;
    const int a = i - L.box.lo[0];
    const int r = (j - L.box.lo[1]) + L.box.dims[1] * (k - L.box.lo[2]);
    const int l = a + L.box.dims[0] * r;
    const int own = colour * (int)L.half + r * L.hx + m;
    const int base = (colour ^ 1) * (int)L.half + r * L.hx;
    const int ry = L.hx, rz = L.hx * L.box.dims[1];
    const uint8_t lab = L.labels[l];
    const T bv = b[own];
    int oxm = base + ((a - 1) >> 1), oxp = base + ((a + 1) >> 1), oym = base - ry + m, oyp = base + ry + m,
        ozm = base - rz + m, ozp = base + rz + m;
    if (L.periodic) {  // the box is the cell: neighbours across the seam
        const int n = L.n;
        if (i == 0) oxm = base + ((n - 1) >> 1);
        if (i == n - 1) oxp = base;
        if (j == 0) oym = base + (n - 1) * ry + m;
        if (j == n - 1) oyp = base - (n - 1) * ry + m;
        if (k == 0) ozm = base + (n - 1) * rz + m;
        if (k == n - 1) ozp = base - (n - 1) * rz + m;
    }
    T zm[3], zp[3];
    zm[0] = load_it<T, S>(z, oxm);
    zp[0] = load_it<T, S>(z, oxp);
    zm[1] = load_it<T, S>(z, oym);
    zp[1] = load_it<T, S>(z, oyp);
    zm[2] = load_it<T, S>(z, ozm);
    zp[2] = load_it<T, S>(z, ozp);
    // keep the loads ahead of the label test (the compiler would otherwise sink
    // them below it and serialise two memory round trips)
    asm volatile("" ::"v"(bv), "v"(zm[0]), "v"(zp[0]), "v"(zm[1]), "v"(zp[1]), "v"(zm[2]), "v"(zp[2]));
    if (!is_unknown(lab)) return;
    T diag, off;
    sw_combine<T, 3>(L, l, lab, zm, zp, &diag, &off);
    if (diag != (T)0) store_t<T, S>(z, own, (bv - off) / diag);
}

template <typename T, typename S, int DIM>
__global__ void __launch_bounds__(256) k_resid_restrict(LevelDev F, LevelDev C, const S* z, const T* b, T* bc) {
    int I = C.core_lo[0] + blockIdx.x * blockDim.x + threadIdx.x;
    int J = C.core_lo[1] + blockIdx.y * blockDim.y + threadIdx.y;
    int K = DIM == 3 ? C.core_lo[2] + blockIdx.z : 0;
    if (I > C.core_hi[0] || J > C.core_hi[1]) return;
    restrict_node<T, S, DIM>(F, C, I, J, K, z, b, bc);
}

template <typename T, typename S, int DIM>
__global__ void __launch_bounds__(256) k_prolong(LevelDev F, LevelDev C, int mode, const S* zc, S* z) {
    int i = F.core_lo[0] + blockIdx.x * blockDim.x + threadIdx.x;
    int j = F.core_lo[1] + blockIdx.y * blockDim.y + threadIdx.y;
    int k = DIM == 3 ? F.core_lo[2] + blockIdx.z : 0;
    if (i > F.core_hi[0] || j > F.core_hi[1]) return;
    prolong_node<T, S, DIM>(F, C, i, j, k, mode, zc, z);
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Index offsets of a level vector for a reference node (i0, j0, k0) with i0, j0
// and k0 even: the node (i0 + ox, j0 + oy, k0 + oz) sits at vidx(i0, j0, k0) +
// voff_even(ox, oy, oz), the same offset for every such reference (its colour
// is that of ox + oy + oz, and the half-index step along x is fixed by the
// parity of lo_x).  boff: the same for the storage box.  Both take only
// uniform values, so the per-load index arithmetic leaves the vector units.
__device__ inline int64_t boff(const Box& b, int ox, int oy, int oz) {
    return (int64_t)ox + (int64_t)b.dims[0] * ((int64_t)oy + (int64_t)b.dims[1] * oz);
}
__device__ inline int64_t voff_even(const LevelDev& L, int ox, int oy, int oz) {
    if (!L.split) return boff(L.box, ox, oy, oz);
    const int lx = L.box.lo[0];
    return (int64_t)((ox + oy + oz) & 1) * L.half + ((int64_t)oy + (int64_t)L.box.dims[1] * oz) * L.hx +
           (((ox - lx) >> 1) - ((-lx) >> 1));
}

// 3D prolongation by coarse cells: the thread of cell (I, J, K) loads the cell's
// eight coarse corners once and corrects the fine nodes 2I + {0,1}, 2J + {0,1},
// 2K + {0,1} (all inside the fine box).  Same parents, weights and summation
// order as prolong_corr.  Every load is issued before the first test.  A cell
// whose far corner lies in the coarse box (INNER: no clamp or wrap) takes its
// indices as per-lane bases plus uniform offsets.
template <typename T, typename S, bool INNER>
__device__ __forceinline__ void prolong_cell(const LevelDev& F, const LevelDev& C, int mode, int I, int J, int K,
                                             const S* zc, S* z) {
    T v[2][2][2];
    uint8_t clab[2][2][2];
    bool inb[2][2][2];
    // INNER: corner (I + a, J + bq, K + cq) at cb[a][colour flip] + its row step
    int64_t cb[2][2] = {{0, 0}, {0, 0}}, clb = 0;
    if (INNER) {
        if (C.split) {
            const int64_t row = ((int64_t)(J - C.box.lo[1]) + (int64_t)C.box.dims[1] * (K - C.box.lo[2])) * C.hx;
            const int par = (I + J + K) & 1;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int f = 0; f < 2; ++f)
                    cb[a][f] = (int64_t)(par ^ f) * C.half + row + ((I + a - C.box.lo[0]) >> 1);
        } else {
            cb[0][0] = cb[0][1] = C.box.idx(I, J, K);
            cb[1][0] = cb[1][1] = cb[0][0] + 1;
        }
        clb = C.box.idx(I, J, K);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bq = 0; bq < 2; ++bq)
#pragma unroll
            for (int cq = 0; cq < 2; ++cq) {
                int64_t ci, li;
                if (INNER) {
                    const int64_t rstep = C.split ? ((int64_t)bq + (int64_t)C.box.dims[1] * cq) * C.hx
                                                  : boff(C.box, 0, bq, cq);
                    ci = cb[a][(a + bq + cq) & 1] + rstep;
                    li = clb + boff(C.box, a, bq, cq);
                    inb[a][bq][cq] = true;
                } else {
                    const int P[3] = {I + a, J + bq, K + cq};
                    int Q[3];
                    bool in = true;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if (C.periodic) {  // coarse parent n_c is the image of 0
                            Q[d] = wrap_near(P[d], C.n);
                        } else {
                            in = in && P[d] >= C.box.lo[d] && P[d] < C.box.lo[d] + C.box.dims[d];
                            Q[d] = clampi(P[d], C.box.lo[d], C.box.lo[d] + C.box.dims[d] - 1);
                        }
                    }
                    inb[a][bq][cq] = in;
                    ci = vidx(C, Q[0], Q[1], Q[2]);
                    li = C.box.idx(Q[0], Q[1], Q[2]);
                }
                v[a][bq][cq] = load_it<T, S>(zc, ci);
                clab[a][bq][cq] = mode == 1 ? C.labels[li] : (uint8_t)0;
            }
    // the fine nodes: 2I, 2J, 2K are even
    const int64_t fb0 = vidx(F, 2 * I, 2 * J, 2 * K), fl0 = F.box.idx(2 * I, 2 * J, 2 * K);
    uint8_t flab[2][2][2];
    T fz[2][2][2];
#pragma unroll
    for (int fc = 0; fc < 2; ++fc)
#pragma unroll
        for (int fb = 0; fb < 2; ++fb)
#pragma unroll
            for (int fa = 0; fa < 2; ++fa) {
                flab[fa][fb][fc] = F.labels[fl0 + boff(F.box, fa, fb, fc)];
                fz[fa][fb][fc] = load_it<T, S>(z, fb0 + voff_even(F, fa, fb, fc));
            }
    asm volatile("" ::"v"(v[0][0][0]), "v"(v[1][1][1]), "v"(fz[0][0][0]), "v"(fz[1][1][1]));
    bool use[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bq = 0; bq < 2; ++bq)
#pragma unroll
            for (int cq = 0; cq < 2; ++cq) {
                const uint8_t kk = clab[a][bq][cq] & KIND_MASK;
                use[a][bq][cq] = mode == 0 || (inb[a][bq][cq] && (kk == K_PLUS || kk == K_MINUS || kk == K_BOX));
                if (!inb[a][bq][cq]) v[a][bq][cq] = 0;
            }
#pragma unroll
    for (int fc = 0; fc < 2; ++fc)
#pragma unroll
        for (int fb = 0; fb < 2; ++fb)
#pragma unroll
            for (int fa = 0; fa < 2; ++fa) {
                const int i = 2 * I + fa, j = 2 * J + fb, k = 2 * K + fc;
                if (i < F.core_lo[0] || i > F.core_hi[0] || j < F.core_lo[1] || j > F.core_hi[1] ||
                    k < F.core_lo[2] || k > F.core_hi[2])
                    continue;
                if (!is_unknown(flab[fa][fb][fc])) continue;
                T sum = 0;
                int cnt = 0;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bq = 0; bq < 2; ++bq)
#pragma unroll
                        for (int cq = 0; cq < 2; ++cq) {
                            if (a > fa || bq > fb || cq > fc) continue;
                            if (use[a][bq][cq]) {
                                sum += v[a][bq][cq];
                                cnt += 1;
                            }
                        }
                if (cnt == 0) continue;
                store_t<T, S>(z, fb0 + voff_even(F, fa, fb, fc), fz[fa][fb][fc] + sum / (T)cnt);
            }
}

// threads over the coarse cells without gaps (nI x nJ x nK, x fastest), blocks
// in XCD-contiguous order
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_prolong_cells(LevelDev F, LevelDev C, int mode, int I0, int J0, int K0,
                                                        int nI, int nJ, int ntot, const S* zc, S* z) {
    const int f = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (f >= ntot) return;
    const int q = f / nI;
    const int I = I0 + (f - q * nI);
    const int J = J0 + q % nJ;
    const int K = K0 + q / nJ;
    const int P[3] = {I, J, K};
    bool inner = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) inner = inner && P[d] >= C.box.lo[d] && P[d] + 1 < C.box.lo[d] + C.box.dims[d];
    if (inner)
        prolong_cell<T, S, true>(F, C, mode, I, J, K, zc, z);
    else
        prolong_cell<T, S, false>(F, C, mode, I, J, K, zc, z);
}

// 3D residual + restriction: the thread of coarse node (I, J, K) evaluates the
// fine residual at c = (2I, 2J, 2K) and its six neighbours from the 25 fine
// values they share, loaded once and all before the first test.  Coordinates
// are clamped into the fine box; a clamped value is only ever used by a node
// that is not an unknown (an unknown's neighbours lie in the box), whose
// residual is zero.  Same weights and summation order as restrict_node.
// INNER: c +- 2 lies in the fine box on every axis (no clamp or wrap), and the
// indices are per-lane bases plus uniform offsets.
template <typename T, typename S, bool INNER>
__device__ __forceinline__ void restrict3_node(const LevelDev& F, const LevelDev& C, int I, int J, int K, const S* z,
                                               const T* b, T* bc, S* zc0) {
    const int c[3] = {2 * I, 2 * J, 2 * K};
    int X[3][5];  // clamped coordinates c[d] - 2 .. c[d] + 2 (not INNER)
    int64_t vb = 0, lb = 0;
    if (INNER) {
        vb = vidx(F, c[0], c[1], c[2]);
        lb = F.box.idx(c[0], c[1], c[2]);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int o = 0; o < 5; ++o)
                X[d][o] = F.periodic ? wrap_near(c[d] + o - 2, F.n)  // the box is the cell
                                     : clampi(c[d] + o - 2, F.box.lo[d], F.box.lo[d] + F.box.dims[d] - 1);
    }
    auto vat = [&](int ox, int oy, int oz) -> int64_t {
        return INNER ? vb + voff_even(F, ox, oy, oz) : vidx(F, X[0][ox + 2], X[1][oy + 2], X[2][oz + 2]);
    };
    auto zat = [&](int ox, int oy, int oz) { return load_it<T, S>(z, vat(ox, oy, oz)); };
    // the seven residual nodes: 0 = c, 1 + 2d = c + e_d, 2 + 2d = c - e_d
    const int off[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    const uint8_t labc = C.labels[C.box.idx(I, J, K)];
    uint8_t lab[7];
    T bv[7], zc[7], zm[7][3], zp[7][3];
    int lbox[7];
#pragma unroll
    for (int n = 0; n < 7; ++n) {
        const int ox = off[n][0], oy = off[n][1], oz = off[n][2];
        lbox[n] = INNER ? (int)(lb + boff(F.box, ox, oy, oz))
                        : (int)F.box.idx(X[0][ox + 2], X[1][oy + 2], X[2][oz + 2]);
        lab[n] = F.labels[lbox[n]];
        bv[n] = b[vat(ox, oy, oz)];
        zc[n] = zat(ox, oy, oz);
        zm[n][0] = zat(ox - 1, oy, oz);
        zp[n][0] = zat(ox + 1, oy, oz);
        zm[n][1] = zat(ox, oy - 1, oz);
        zp[n][1] = zat(ox, oy + 1, oz);
        zm[n][2] = zat(ox, oy, oz - 1);
        zp[n][2] = zat(ox, oy, oz + 1);
    }
    asm volatile("" ::"v"(bv[0]), "v"(zc[0]), "v"(zm[1][0]), "v"(zp[2][0]), "v"(zm[5][2]), "v"(zp[6][2]));
    const int64_t vc = vidx(C, I, J, K);
    bool inside = is_unknown(labc);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        inside = inside && (INNER || F.periodic || (c[d] - 1 >= F.box.lo[d] && c[d] + 1 < F.box.lo[d] + F.box.dims[d]));
    if (!inside) {
        bc[vc] = (T)0;
        if (zc0) store_t<T, S>(zc0, vc, (T)0);
        return;
    }
    T r[7];
#pragma unroll
    for (int n = 0; n < 7; ++n) {
        r[n] = (T)0;
        if (is_unknown(lab[n])) {
            T diag, offd;
            sw_combine<T, 3>(F, lbox[n], lab[n], zm[n], zp[n], &diag, &offd);
            r[n] = bv[n] - (diag * zc[n] + offd);
        }
    }
    const T w0 = (T)0.5, w1 = (T)(1.0 / 12.0);
    T acc = w0 * r[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) acc += w1 * (r[1 + 2 * d] + r[2 + 2 * d]);
    const T bval = (T)4 * acc;
    bc[vc] = bval;
    if (zc0) {
        // the coarse level's first half-sweep (colour 0) from a zero iterate: the
        // neighbours are zero, so z = b / diag at colour-0 unknowns and 0 elsewhere
        T zv = (T)0;
        if (((I + J + K) & 1) == 0) {
            const T diag = (labc & F_SW_IRR) ? rec_ptr<T>(C)[(int64_t)C.irr_index[C.box.idx(I, J, K)] * 7] : (T)(-6);
            if (diag != (T)0) zv = bval / diag;
        }
        store_t<T, S>(zc0, vc, zv);
    }
}

template <typename T, typename S>
__global__ void __launch_bounds__(256) k_restrict3(LevelDev F, LevelDev C, int gx, int gy, const S* z, const T* b,
                                                    T* bc, S* zc0) {
    const Blk3 B = xcd_block3(gx, gy);
    const int I = C.core_lo[0] + B.x * 64 + (threadIdx.x & 63);
    const int J = C.core_lo[1] + B.y * 4 + (threadIdx.x >> 6);
    const int K = C.core_lo[2] + B.z;
    if (I > C.core_hi[0] || J > C.core_hi[1] || K > C.core_hi[2]) return;
    const int c[3] = {2 * I, 2 * J, 2 * K};
    bool inner = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) inner = inner && c[d] - 2 >= F.box.lo[d] && c[d] + 2 < F.box.lo[d] + F.box.dims[d];
    if (inner)
        restrict3_node<T, S, true>(F, C, I, J, K, z, b, bc, zc0);
    else
        restrict3_node<T, S, false>(F, C, I, J, K, z, b, bc, zc0);
}

// The first steps of the level-0 pre-smoothing of a colour-split level in one
// pass: the cast of the FP64 input (as run_cast_in), the zero iterate and the
// colour-0 half-sweep from it (z = b / diag at colour-0 unknowns: every
// neighbour is zero).  A thread owns the two nodes 2m, 2m + 1 of a box row (one
// of each colour); every row of the box is covered, padding entries included.
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_cast_sweep0(LevelDev L, const double* v, const double* scale, double h2,
                                                     double bp, double bm, T* b, S* z) {
    // threads over (box row, pair) without gaps: f = r hx + m
    const int f = blockIdx.x * 256 + threadIdx.x;
    const int r = f / L.hx, m = f - r * L.hx;
    const int nrows = L.box.dims[1] * L.box.dims[2];
    if (r >= nrows) return;
    const int j = L.box.lo[1] + r % L.box.dims[1], k = L.box.lo[2] + r / L.box.dims[1];
    const int par = (L.box.lo[0] + j + k) & 1;  // colour of node a = 2m
    const double sc = *scale;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int a = 2 * m + q, colour = par ^ q;
        const int64_t e = (int64_t)colour * L.half + (int64_t)r * L.hx + m;
        double val = 0.0;
        uint8_t lab = 0;
        int64_t l = 0;
        if (a < L.box.dims[0]) {
            l = (int64_t)a + (int64_t)L.box.dims[0] * r;
            lab = L.labels[l];
            const uint8_t kk = lab & KIND_MASK;
            if (kk == K_PLUS) val = sc * h2 * v[l] / bp;
            else if (kk == K_MINUS) val = sc * h2 * v[l] / bm;
        }
        const T bv = (T)val;
        b[e] = bv;
        T zv = (T)0;
        if (colour == 0 && is_unknown(lab)) {
            const T diag = (lab & F_SW_IRR) ? rec_ptr<T>(L)[(int64_t)L.irr_index[l] * 7] : (T)(-6);
            if (diag != (T)0) zv = bv / diag;
        }
        store_t<T, S>(z, e, zv);
    }
}

// The last level-0 post-smoothing half-sweep (colour 1) of a colour-split level
// writing the V-cycle's FP64 output instead of z (as run_cast_out: z / scale at
// unknowns, 0 elsewhere) for both nodes of each pair 2m, 2m + 1 of the core's
// rows.  The output is zero off those rows already (a Krylov basis column).
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_rbgs_split_out(LevelDev L, int ny, int nrows, const S* z, const T* b,
                                                        double* out, const double* scale) {
    // threads over (core row, pair) without gaps, blocks in XCD-contiguous order
    const int f = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int crow = f / L.hx;
    if (crow >= nrows) return;
    const int m = f - crow * L.hx;
    const int j = L.core_lo[1] + crow % ny;
    const int k = L.core_lo[2] + crow / ny;
    const int p1 = (1 ^ (L.box.lo[0] + j + k)) & 1;
    const int a1 = 2 * m + p1, a0 = 2 * m + (p1 ^ 1);  // colour-1 node and its colour-0 partner
    const int r = (j - L.box.lo[1]) + L.box.dims[1] * (k - L.box.lo[2]);
    const int row = L.box.dims[0] * r;
    const double inv = 1.0 / *scale;
    if (a0 < L.box.dims[0]) {
        const uint8_t lab0 = L.labels[row + a0];
        out[row + a0] = is_unknown(lab0) ? (double)load_it<T, S>(z, r * L.hx + m) * inv : 0.0;
    }
    if (a1 >= L.box.dims[0]) return;
    const int i = L.box.lo[0] + a1;
    const uint8_t lab = L.labels[row + a1];
    double o = 0.0;
    if (i >= L.core_lo[0] && i <= L.core_hi[0] && is_unknown(lab)) {
        const int own = (int)L.half + r * L.hx + m;
        const int ry = L.hx, rz = L.hx * L.box.dims[1];
        const int base = r * L.hx;  // colour-0 array, row r
        int oxm = base + ((a1 - 1) >> 1), oxp = base + ((a1 + 1) >> 1), oym = base - ry + m, oyp = base + ry + m,
            ozm = base - rz + m, ozp = base + rz + m;
        if (L.periodic) {  // the box is the cell: neighbours across the seam
            const int n = L.n;
            if (i == 0) oxm = base + ((n - 1) >> 1);
            if (i == n - 1) oxp = base;
            if (j == 0) oym = base + (n - 1) * ry + m;
            if (j == n - 1) oyp = base - (n - 1) * ry + m;
            if (k == 0) ozm = base + (n - 1) * rz + m;
            if (k == n - 1) ozp = base - (n - 1) * rz + m;
        }
        T zm[3], zp[3];
        zm[0] = load_it<T, S>(z, oxm);
        zp[0] = load_it<T, S>(z, oxp);
        zm[1] = load_it<T, S>(z, oym);
        zp[1] = load_it<T, S>(z, oyp);
        zm[2] = load_it<T, S>(z, ozm);
        zp[2] = load_it<T, S>(z, ozp);
        const T bv = b[own];
        T diag, off;
        sw_combine<T, 3>(L, row + a1, lab, zm, zp, &diag, &off);
        const T zn = diag != (T)0 ? round_s<T, S>((bv - off) / diag) : load_it<T, S>(z, own);
        o = (double)zn * inv;
    }
    out[row + a1] = o;
}

template <typename T, typename S>
__global__ void k_coarse_solve(const int32_t* list, int64_t nc, const T* Ainv, const T* b, S* z) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= nc) return;
    coarse_row<T, S>(list, nc, Ainv, b, z, r);
}

// ---- the small levels of a V-cycle in one workgroup: levels first..last of the
// device table, coarse solve included; barriers separate the phases.
template <int DIM, typename F>
__device__ inline void for_core(const LevelDev& L, F fn) {
    const int nx = L.core_hi[0] - L.core_lo[0] + 1, ny = L.core_hi[1] - L.core_lo[1] + 1;
    const int nz = DIM == 3 ? L.core_hi[2] - L.core_lo[2] + 1 : 1;
    if (nx <= 0 || ny <= 0 || nz <= 0) return;
    const int64_t tot = (int64_t)nx * ny * nz;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
        int i = L.core_lo[0] + (int)(t % nx);
        int j = L.core_lo[1] + (int)((t / nx) % ny);
        int k = DIM == 3 ? L.core_lo[2] + (int)(t / ((int64_t)nx * ny)) : 0;
        fn(i, j, k);
    }
}

template <typename T, typename S, int DIM>
__device__ inline void tail_body(const TailDev& D) {
    for (int l = D.first; l < D.last; ++l) {
        const LevelDev& L = D.lev[l];
        S* z = (S*)D.z[l];
        const T* b = (const T*)D.b[l];
        for (int64_t t = threadIdx.x; t < L.box.size(); t += blockDim.x) z[t] = S(0.0f);
        __syncthreads();
        for (int s = 0; s < D.nu_pre; ++s)
            for (int c = 0; c < 2; ++c) {
                for_core<DIM>(L, [&](int i, int j, int k) { rbgs_node<T, S, DIM>(L, i, j, k, c, z, b); });
                __syncthreads();
            }
        const LevelDev& C = D.lev[l + 1];
        T* bc = (T*)D.b[l + 1];
        for_core<DIM>(C, [&](int i, int j, int k) { restrict_node<T, S, DIM>(L, C, i, j, k, z, b, bc); });
        __syncthreads();
    }
    {
        const LevelDev& L = D.lev[D.last];
        S* z = (S*)D.z[D.last];
        for (int64_t t = threadIdx.x; t < L.box.size(); t += blockDim.x) z[t] = S(0.0f);
        __syncthreads();
        for (int64_t r = threadIdx.x; r < D.nc; r += blockDim.x)
            coarse_row<T, S>(D.clist, D.nc, (const T*)D.Ainv, (const T*)D.b[D.last], z, r);
        __syncthreads();
    }
    for (int l = D.last - 1; l >= D.first; --l) {
        const LevelDev& L = D.lev[l];
        const LevelDev& C = D.lev[l + 1];
        S* z = (S*)D.z[l];
        const S* zc = (const S*)D.z[l + 1];
        const T* b = (const T*)D.b[l];
        for_core<DIM>(L, [&](int i, int j, int k) { prolong_node<T, S, DIM>(L, C, i, j, k, D.mode, zc, z); });
        __syncthreads();
        for (int s = 0; s < D.nu_post; ++s)
            for (int c = 0; c < 2; ++c) {
                for_core<DIM>(L, [&](int i, int j, int k) { rbgs_node<T, S, DIM>(L, i, j, k, c, z, b); });
                __syncthreads();
            }
    }
}

// The same tail with every vector of its levels in LDS: b of the first tail
// level is copied in, the cycle over the tail levels runs on LDS arrays (labels
// and Shortley-Weller rows are read from global memory, where they stay
// cached), and z of the first tail level is copied out for the prolongation
// onto the finer level.  The vectors of level l start at byte D.lds_z[l] and
// D.lds_b[l] of the dynamic LDS area.
template <typename T, typename S, int DIM>
__device__ inline void tail_lds_body(const TailDev& D, char* tail_smem) {
    auto zl = [&](int l) { return (S*)(tail_smem + D.lds_z[l]); };
    auto bl = [&](int l) { return (T*)(tail_smem + D.lds_b[l]); };
    {
        const int64_t n0 = D.lev[D.first].box.size();
        const T* bg = (const T*)D.b[D.first];
        for (int64_t t = threadIdx.x; t < n0; t += blockDim.x) bl(D.first)[t] = bg[t];
        for (int l = D.first + 1; l <= D.last; ++l)
            for (int64_t t = threadIdx.x; t < D.lev[l].box.size(); t += blockDim.x) bl(l)[t] = (T)0;
    }
    for (int l = D.first; l < D.last; ++l) {
        const LevelDev& L = D.lev[l];
        S* z = zl(l);
        const T* b = bl(l);
        for (int64_t t = threadIdx.x; t < L.box.size(); t += blockDim.x) z[t] = S(0.0f);
        __syncthreads();
        for (int s = 0; s < D.nu_pre; ++s)
            for (int c = 0; c < 2; ++c) {
                for_core<DIM>(L, [&](int i, int j, int k) { rbgs_node<T, S, DIM>(L, i, j, k, c, z, b); });
                __syncthreads();
            }
        const LevelDev& C = D.lev[l + 1];
        T* bc = bl(l + 1);
        for_core<DIM>(C, [&](int i, int j, int k) { restrict_node<T, S, DIM>(L, C, i, j, k, z, b, bc); });
        __syncthreads();
    }
    {
        const LevelDev& L = D.lev[D.last];
        S* z = zl(D.last);
        for (int64_t t = threadIdx.x; t < L.box.size(); t += blockDim.x) z[t] = S(0.0f);
        __syncthreads();
        for (int64_t r = threadIdx.x; r < D.nc; r += blockDim.x)
            coarse_row<T, S>(D.clist, D.nc, (const T*)D.Ainv, bl(D.last), z, r);
        __syncthreads();
    }
    for (int l = D.last - 1; l >= D.first; --l) {
        const LevelDev& L = D.lev[l];
        const LevelDev& C = D.lev[l + 1];
        S* z = zl(l);
        const S* zc = zl(l + 1);
        const T* b = bl(l);
        for_core<DIM>(L, [&](int i, int j, int k) { prolong_node<T, S, DIM>(L, C, i, j, k, D.mode, zc, z); });
        __syncthreads();
        for (int s = 0; s < D.nu_post; ++s)
            for (int c = 0; c < 2; ++c) {
                for_core<DIM>(L, [&](int i, int j, int k) { rbgs_node<T, S, DIM>(L, i, j, k, c, z, b); });
                __syncthreads();
            }
    }
    {
        const int64_t n0 = D.lev[D.first].box.size();
        S* zg = (S*)D.z[D.first];
        for (int64_t t = threadIdx.x; t < n0; t += blockDim.x) zg[t] = zl(D.first)[t];
    }
}

template <typename T, typename S, int DIM>
__global__ void __launch_bounds__(1024) k_tail(const TailDev* __restrict__ Dp) {
    tail_body<T, S, DIM>(*Dp);
}

template <typename T, typename S, int DIM>
__global__ void __launch_bounds__(1024) k_tail_lds(const TailDev* __restrict__ Dp) {
    extern __shared__ __align__(16) char tail_smem[];
    tail_lds_body<T, S, DIM>(*Dp, tail_smem);
}

// The tails of several independent problems in one launch, one workgroup per
// problem: workgroup q runs exactly the single-problem tail of B.d[q] (its LDS
// form when B.lds[q] > 0), so each problem's result is bit-for-bit the one of
// its own launch.
template <typename T, typename S, int DIM>
__global__ void __launch_bounds__(1024) k_tail_batch(TailBatch B) {
    extern __shared__ __align__(16) char tail_smem[];
    const int q = blockIdx.x;
    if (q >= B.count) return;
    if (B.lds[q] > 0)
        tail_lds_body<T, S, DIM>(*B.d[q], tail_smem);
    else
        tail_body<T, S, DIM>(*B.d[q]);
}

// ---- fused 2D smoothing legs with LDS tiles -------------------------------------
// Each workgroup owns a TX x TY tile of the level's core and loads it with a halo
// of HALO nodes.  A red-black half-sweep invalidates one more ring of the loaded
// region, so after nh <= HALO - 2 half-sweeps the tile interior and one ring
// around it are exact: the interior is identical to global red-black
// Gauss-Seidel, and the residual is exact on the footprint of every coarse node
// whose centre 2I lies in the tile.  Iterates are rounded to the storage type
// after every update, as the unfused kernels do.
// The load phase issues every global load of a thread before using any of them
// (labels, b, z and record indices are read unconditionally inside the box), and
// caches the Shortley-Weller rows of the tile's irregular nodes in LDS.
constexpr int FTX = 32, FTY = 32, FHALO = 6;
constexpr int FLX = FTX + 2 * FHALO, FLY = FTY + 2 * FHALO;
constexpr int FN = FLX * FLY;
constexpr int FTHREADS = 1024;
constexpr int FNPT = (FN + FTHREADS - 1) / FTHREADS;
constexpr int FREC = 320;  // irregular rows cached per tile
constexpr int FCX = FLX / 2 + 2, FCY = FLY / 2 + 2;  // coarse parents of the loaded region


template <typename T>
struct FusedLDS {
    T zs[FLY][FLX];
    T bs[FLY][FLX];
    uint8_t ls[FLY][FLX];
    int16_t slot[FLY][FLX];  // >= 0: cached row; -1 regular; -2 irregular, row read from global
    T rec[FREC][5];
    int nrec;
};

// the FP64 input of a V-cycle and its scaling (run_cast_in), for the first leg
template <typename T>
struct CastInT {
    const double* v = nullptr;
    const double* scale = nullptr;
    double h2 = 0, bp = 1, bm = 1;
    T* b_out = nullptr;
};

template <typename T>
__device__ inline void lds_row(const LevelDev& L, const FusedLDS<T>& S, int i, int j, int lx, int ly, T* acc,
                               T* diag) {
    const uint8_t lab = S.ls[ly][lx];
    if (!(lab & F_SW_IRR)) {
        T a = (T)0;
        a += S.zs[ly][lx + 1] + S.zs[ly][lx - 1];
        a += S.zs[ly + 1][lx] + S.zs[ly - 1][lx];
        *acc = a;
        *diag = (T)(-4);
        return;
    }
    const int sl = S.slot[ly][lx];
    const T* rec = sl >= 0 ? S.rec[sl] : rec_ptr<T>(L) + (int64_t)L.irr_index[L.box.idx(i, j, 0)] * 5;
    T a = (T)0;
    a += rec[1] * S.zs[ly][lx - 1] + rec[2] * S.zs[ly][lx + 1];
    a += rec[3] * S.zs[ly - 1][lx] + rec[4] * S.zs[ly + 1][lx];
    *acc = a;
    *diag = rec[0];
}

// one half-sweep over the loaded region (outer ring skipped: its neighbours are not loaded)
template <typename T, typename S>
__device__ inline void lds_half_sweep(const LevelDev& L, int x0, int y0, int colour, FusedLDS<T>& Sh) {
    for (int t = threadIdx.x; t < (FLX - 2) * (FLY - 2); t += FTHREADS) {
        const int lx = 1 + t % (FLX - 2), ly = 1 + t / (FLX - 2);
        const int i = x0 - FHALO + lx, j = y0 - FHALO + ly;
        if (((i + j) & 1) != colour) continue;
        if (!is_unknown(Sh.ls[ly][lx])) continue;
        T acc, diag;
        lds_row<T>(L, Sh, i, j, lx, ly, &acc, &diag);
        if (diag != (T)0) Sh.zs[ly][lx] = round_s<T, S>((Sh.bs[ly][lx] - acc) / diag);
    }
}

template <typename T>
__device__ inline T lds_resid(const LevelDev& L, const FusedLDS<T>& Sh, int i, int j, int lx, int ly) {
    if (!is_unknown(Sh.ls[ly][lx])) return (T)0;
    T acc, diag;
    lds_row<T>(L, Sh, i, j, lx, ly, &acc, &diag);
    return Sh.bs[ly][lx] - (diag * Sh.zs[ly][lx] + acc);
}

// load labels, b, z (optional) and the irregular rows of the tile into LDS.
// With C.v set, b is made from the FP64 vector instead (as run_cast_in does)
// and the tile's own nodes of it are written to b for the later legs.
template <typename T, typename S>
__device__ inline void lds_load(const LevelDev& F, int x0, int y0, const S* z, const T* b, FusedLDS<T>& Sh,
                                const CastInT<T>& C = CastInT<T>{}) {
    uint8_t labv[FNPT];
    T bv[FNPT], zv[FNPT];
    int32_t irr[FNPT];
    if (threadIdx.x == 0) Sh.nrec = 0;
#pragma unroll
    for (int q = 0; q < FNPT; ++q) {
        const int t = threadIdx.x + FTHREADS * q;
        const int lx = t % FLX, ly = t / FLX;
        const int i = x0 - FHALO + lx, j = y0 - FHALO + ly;
        const bool inb = t < FN && i >= F.box.lo[0] && i < F.box.lo[0] + F.box.dims[0] && j >= F.box.lo[1] &&
                         j < F.box.lo[1] + F.box.dims[1];
        const int64_t l = inb ? F.box.idx(i, j, 0) : 0;
        labv[q] = inb ? F.labels[l] : (uint8_t)0;
        if (C.v) {
            double val = 0.0;
            if (inb) {
                const uint8_t kk = labv[q] & KIND_MASK;
                const double vl = C.v[l], sc = *C.scale;
                if (kk == K_PLUS) val = sc * C.h2 * vl / C.bp;
                else if (kk == K_MINUS) val = sc * C.h2 * vl / C.bm;
            }
            bv[q] = (T)val;
            if (inb && lx >= FHALO && lx < FHALO + FTX && ly >= FHALO && ly < FHALO + FTY)
                C.b_out[l] = bv[q];  // this tile's nodes: each written by one tile
        } else {
            bv[q] = inb ? b[l] : (T)0;
        }
        zv[q] = (inb && z) ? load_it<T, S>(z, l) : (T)0;
        irr[q] = inb ? F.irr_index[l] : -1;
    }
    __syncthreads();  // nrec = 0 visible
#pragma unroll
    for (int q = 0; q < FNPT; ++q) {
        const int t = threadIdx.x + FTHREADS * q;
        if (t >= FN) continue;
        const int lx = t % FLX, ly = t / FLX;
        const bool unk = is_unknown(labv[q]);
        Sh.ls[ly][lx] = labv[q];
        Sh.bs[ly][lx] = unk ? bv[q] : (T)0;
        Sh.zs[ly][lx] = unk ? zv[q] : (T)0;
        int sl = -1;
        if (unk && (labv[q] & F_SW_IRR)) {
            sl = atomicAdd(&Sh.nrec, 1);
            if (sl < FREC) {
                const T* rec = rec_ptr<T>(F) + (int64_t)irr[q] * 5;
#pragma unroll
                for (int r = 0; r < 5; ++r) Sh.rec[sl][r] = rec[r];
            } else {
                sl = -2;
            }
        }
        Sh.slot[ly][lx] = (int16_t)sl;
    }
}

// coarse parents of the loaded region: fetched into registers first (so the
// loads overlap the tile's own), then staged in LDS
constexpr int FCPT = (FCX * FCY + FTHREADS - 1) / FTHREADS;
template <typename T, typename S>
__device__ inline void prolong_fetch(const LevelDev& C, const S* zc, int x0, int y0, T (&cv)[FCPT],
                                     uint8_t (&clv)[FCPT]) {
    const int cx0 = (x0 - FHALO) >> 1, cy0 = (y0 - FHALO) >> 1;
    constexpr int CN = FCX * FCY;
#pragma unroll
    for (int q = 0; q < FCPT; ++q) {
        const int t = threadIdx.x + FTHREADS * q;
        const int P0 = cx0 + t % FCX, P1 = cy0 + t / FCX;
        const bool cin = t < CN && P0 >= C.box.lo[0] && P0 < C.box.lo[0] + C.box.dims[0] && P1 >= C.box.lo[1] &&
                         P1 < C.box.lo[1] + C.box.dims[1];
        const int64_t lp = cin ? C.box.idx(P0, P1, 0) : 0;
        cv[q] = cin ? load_it<T, S>(zc, lp) : (T)0;
        clv[q] = cin ? C.labels[lp] : (uint8_t)255;  // 255: outside the coarse box
    }
}

// z += P zc on the loaded region (as prolong_node), the coarse parents staged in LDS
template <typename T, typename S>
__device__ inline void lds_prolong(int mode, int x0, int y0, FusedLDS<T>& Sh, const T (&cv)[FCPT],
                                   const uint8_t (&clv)[FCPT], T (*cz)[FCX], uint8_t (*cl)[FCX]) {
    const int cx0 = (x0 - FHALO) >> 1, cy0 = (y0 - FHALO) >> 1;
    constexpr int CN = FCX * FCY;
#pragma unroll
    for (int q = 0; q < FCPT; ++q) {
        const int t = threadIdx.x + FTHREADS * q;
        if (t < CN) {
            cz[t / FCX][t % FCX] = cv[q];
            cl[t / FCX][t % FCX] = clv[q];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < FN; t += FTHREADS) {
        const int lx = t % FLX, ly = t / FLX;
        if (!is_unknown(Sh.ls[ly][lx])) continue;
        const int i = x0 - FHALO + lx, j = y0 - FHALO + ly;
        const int lo0 = i >> 1, lo1 = j >> 1;
        const int nb0 = (i & 1) ? 2 : 1, nb1 = (j & 1) ? 2 : 1;
        T sum = 0;
        int cnt = 0;
        for (int a = 0; a < nb0; ++a)
            for (int bq = 0; bq < nb1; ++bq) {
                const int P0 = lo0 + a - cx0, P1 = lo1 + bq - cy0;
                const uint8_t kk = cl[P1][P0];
                const bool cin = kk != 255;
                T v = cin ? cz[P1][P0] : (T)0;
                bool use = mode == 0;
                if (mode == 1) {
                    const uint8_t k2 = kk & KIND_MASK;
                    use = cin && (k2 == K_PLUS || k2 == K_MINUS || k2 == K_BOX);
                }
                if (use) {
                    sum += v;
                    cnt += 1;
                }
            }
        if (cnt > 0) Sh.zs[ly][lx] = round_s<T, S>(Sh.zs[ly][lx] + sum / (T)cnt);
    }
}

template <typename T, typename S>
__device__ inline void lds_store(const LevelDev& F, int x0, int y0, const FusedLDS<T>& Sh, S* z) {
    for (int t = threadIdx.x; t < FTX * FTY; t += FTHREADS) {
        const int lx = FHALO + t % FTX, ly = FHALO + t / FTX;
        const int i = x0 - FHALO + lx, j = y0 - FHALO + ly;
        if (i > F.core_hi[0] || j > F.core_hi[1]) continue;
        if (is_unknown(Sh.ls[ly][lx])) store_t<T, S>(z, F.box.idx(i, j, 0), Sh.zs[ly][lx]);
    }
}

// the tile's core nodes as the V-cycle's FP64 output (as run_cast_out does:
// out = z / scale at unknowns, 0 elsewhere; nodes outside the core untouched)
template <typename T, typename S>
__device__ inline void lds_store_out(const LevelDev& F, int x0, int y0, const FusedLDS<T>& Sh, double* out,
                                     const double* scale) {
    const double inv = 1.0 / *scale;
    for (int t = threadIdx.x; t < FTX * FTY; t += FTHREADS) {
        const int lx = FHALO + t % FTX, ly = FHALO + t / FTX;
        const int i = x0 - FHALO + lx, j = y0 - FHALO + ly;
        if (i > F.core_hi[0] || j > F.core_hi[1]) continue;
        out[F.box.idx(i, j, 0)] = is_unknown(Sh.ls[ly][lx]) ? (double)Sh.zs[ly][lx] * inv : 0.0;
    }
}

// down leg: z = 0, nh half-sweeps (red first), write z, then bc = 4 HW(residual)
template <typename T, typename S>
__global__ void __launch_bounds__(FTHREADS) k_down_2d(LevelDev F, LevelDev C, const T* __restrict__ b,
                                                      S* __restrict__ z, T* __restrict__ bc, int nh, CastInT<T> cin) {
    __shared__ FusedLDS<T> Sh;
    const int x0 = F.core_lo[0] + blockIdx.x * FTX, y0 = F.core_lo[1] + blockIdx.y * FTY;
    // coarse nodes whose centre 2I lies in this tile (at most FTX/2 x FTY/2 <= FTHREADS);
    // their labels are fetched with the tile's loads
    const int I0 = (x0 + 1) >> 1, J0 = (y0 + 1) >> 1;
    const int I1 = (min(x0 + FTX - 1, F.core_hi[0])) >> 1, J1 = (min(y0 + FTY - 1, F.core_hi[1])) >> 1;
    const int nI = I1 - I0 + 1, nJ = J1 - J0 + 1;
    const int tI = I0 + (int)threadIdx.x % max(nI, 1), tJ = J0 + (int)threadIdx.x / max(nI, 1);
    const bool mine = (int)threadIdx.x < nI * nJ && tI >= C.core_lo[0] && tI <= C.core_hi[0] &&
                      tJ >= C.core_lo[1] && tJ <= C.core_hi[1];
    const uint8_t clab = mine ? C.labels[C.box.idx(tI, tJ, 0)] : (uint8_t)0;
    lds_load<T, S>(F, x0, y0, nullptr, b, Sh, cin);
    __syncthreads();
    for (int h2 = 0; h2 < nh; ++h2) {
        lds_half_sweep<T, S>(F, x0, y0, h2 & 1, Sh);
        __syncthreads();
    }
    lds_store<T, S>(F, x0, y0, Sh, z);
    const T w0 = (T)0.5, w1 = (T)0.125;
    if (mine) {
        const int I = tI, J = tJ;
        const int64_t lc = C.box.idx(I, J, 0);
        if (!is_unknown(clab)) {
            bc[lc] = (T)0;
            return;
        }
        const int fi = 2 * I, fj = 2 * J;
        const int lx = fi - (x0 - FHALO), ly = fj - (y0 - FHALO);
        T acc = w0 * lds_resid<T>(F, Sh, fi, fj, lx, ly);
        acc += w1 * (lds_resid<T>(F, Sh, fi + 1, fj, lx + 1, ly) + lds_resid<T>(F, Sh, fi - 1, fj, lx - 1, ly));
        acc += w1 * (lds_resid<T>(F, Sh, fi, fj + 1, lx, ly + 1) + lds_resid<T>(F, Sh, fi, fj - 1, lx, ly - 1));
        bc[lc] = (T)4 * acc;
    }
}

// up leg: z_out = smoothed (z_in + P zc), nh half-sweeps (red first).  z_in and
// z_out are distinct: a tile's halo is read from z_in while neighbouring tiles
// write their results, so the result does not depend on block timing.
template <typename T, typename S>
__global__ void __launch_bounds__(FTHREADS) k_up_2d(LevelDev F, LevelDev C, int mode, const S* __restrict__ zc,
                                                    const T* __restrict__ b, const S* __restrict__ z_in,
                                                    S* __restrict__ z, int nh, double* __restrict__ out,
                                                    const double* __restrict__ out_scale) {
    __shared__ FusedLDS<T> Sh;
    __shared__ T cz[FCY][FCX];
    __shared__ uint8_t cl[FCY][FCX];
    const int x0 = F.core_lo[0] + blockIdx.x * FTX, y0 = F.core_lo[1] + blockIdx.y * FTY;
    T cv[FCPT];
    uint8_t clv[FCPT];
    prolong_fetch<T, S>(C, zc, x0, y0, cv, clv);
    lds_load<T, S>(F, x0, y0, z_in, b, Sh);
    lds_prolong<T, S>(mode, x0, y0, Sh, cv, clv, cz, cl);
    __syncthreads();
    for (int h2 = 0; h2 < nh; ++h2) {
        lds_half_sweep<T, S>(F, x0, y0, h2 & 1, Sh);
        __syncthreads();
    }
    if (out)
        lds_store_out<T, S>(F, x0, y0, Sh, out, out_scale);
    else
        lds_store<T, S>(F, x0, y0, Sh, z);
}

template <typename T, typename S>
bool run_down_fused(const LevelDev& F, const LevelDev& C, const T* b, S* z, T* bc, int nu, hipStream_t s,
                    const CastInArgs* cast) {
    if (F.dim != 2 || 2 * nu > FHALO - 2) return false;
    const int nx = F.core_hi[0] - F.core_lo[0] + 1, ny = F.core_hi[1] - F.core_lo[1] + 1;
    if (nx <= 0 || ny <= 0) return false;
    CastInT<T> cin;
    if (cast) {
        cin.v = cast->v;
        cin.scale = cast->scale;
        cin.h2 = cast->h2;
        cin.bp = cast->bp;
        cin.bm = cast->bm;
        cin.b_out = const_cast<T*>(b);
    }
    hipLaunchKernelGGL((k_down_2d<T, S>), dim3(cdiv(nx, FTX), cdiv(ny, FTY)), dim3(FTHREADS), 0, s, F, C, b, z, bc,
                       2 * nu, cin);
    IIM_LAUNCH_CHECK();
    return true;
}

template <typename T, typename S>
bool run_up_fused(const LevelDev& F, const LevelDev& C, int mode, const S* zc, const T* b, const S* z_in, S* z_out,
                  int nu, hipStream_t s, double* out, const double* out_scale) {
    if (F.dim != 2 || 2 * nu > FHALO - 2) return false;
    if ((const void*)z_in == (const void*)z_out) throw Error(IIM_E_INTERNAL, "fused up leg needs distinct buffers");
    const int nx = F.core_hi[0] - F.core_lo[0] + 1, ny = F.core_hi[1] - F.core_lo[1] + 1;
    if (nx <= 0 || ny <= 0) return false;
    hipLaunchKernelGGL((k_up_2d<T, S>), dim3(cdiv(nx, FTX), cdiv(ny, FTY)), dim3(FTHREADS), 0, s, F, C, mode, zc, b,
                       z_in, z_out, 2 * nu, out, out_scale);
    IIM_LAUNCH_CHECK();
    return true;
}

template <typename T, typename S>
void run_tail(int dim, const TailDev* d_tail, int64_t lds_bytes, hipStream_t s) {
    if (lds_bytes > 0) {
        if (lds_bytes > TAIL_LDS_MAX) throw Error(IIM_E_INTERNAL, "tail: LDS request too large");
        if (dim == 2)
            hipLaunchKernelGGL((k_tail_lds<T, S, 2>), dim3(1), dim3(1024), (unsigned)lds_bytes, s, d_tail);
        else
            hipLaunchKernelGGL((k_tail_lds<T, S, 3>), dim3(1), dim3(1024), (unsigned)lds_bytes, s, d_tail);
    } else if (dim == 2) {
        hipLaunchKernelGGL((k_tail<T, S, 2>), dim3(1), dim3(1024), 0, s, d_tail);
    } else {
        hipLaunchKernelGGL((k_tail<T, S, 3>), dim3(1), dim3(1024), 0, s, d_tail);
    }
    IIM_LAUNCH_CHECK();
}

template <typename T, typename S>
void run_tail_batch(int dim, const TailBatch& B, hipStream_t s) {
    if (B.count <= 0) return;
    if (B.count > TAIL_BATCH_MAX) throw Error(IIM_E_INTERNAL, "tail batch too large");
    int64_t lds = 0;
    for (int q = 0; q < B.count; ++q) lds = std::max(lds, B.lds[q]);
    if (lds > TAIL_LDS_MAX) throw Error(IIM_E_INTERNAL, "tail: LDS request too large");
    if (dim == 2)
        hipLaunchKernelGGL((k_tail_batch<T, S, 2>), dim3(B.count), dim3(1024), (unsigned)lds, s, B);
    else
        hipLaunchKernelGGL((k_tail_batch<T, S, 3>), dim3(B.count), dim3(1024), (unsigned)lds, s, B);
    IIM_LAUNCH_CHECK();
}

// lets every LDS-resident tail instantiation request TAIL_LDS_MAX bytes (once per process)
void enable_tail_lds() {
    static std::once_flag once;
    std::call_once(once, [] {
        const void* fns[] = {(const void*)k_tail_lds<double, double, 2>, (const void*)k_tail_lds<double, double, 3>,
                             (const void*)k_tail_lds<float, float, 2>,   (const void*)k_tail_lds<float, float, 3>,
                             (const void*)k_tail_lds<float, __half, 2>,  (const void*)k_tail_lds<float, __half, 3>,
                             (const void*)k_tail_batch<double, double, 2>, (const void*)k_tail_batch<double, double, 3>,
                             (const void*)k_tail_batch<float, float, 2>,   (const void*)k_tail_batch<float, float, 3>,
                             (const void*)k_tail_batch<float, __half, 2>,  (const void*)k_tail_batch<float, __half, 3>};
        for (const void* f : fns)
            IIM_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TAIL_LDS_MAX));
    });
}

template <typename S>
__global__ void k_zero(S* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = S(0.0f);
}

static inline void level_grid(const LevelDev& L, dim3* grd, dim3* blk) {
    int nx = L.core_hi[0] - L.core_lo[0] + 1, ny = L.core_hi[1] - L.core_lo[1] + 1;
    int nz = L.dim == 3 ? L.core_hi[2] - L.core_lo[2] + 1 : 1;
    *blk = dim3(64, 4, 1);
    *grd = dim3(cdiv(std::max(nx, 1), 64), cdiv(std::max(ny, 1), 4), std::max(nz, 1));
}

template <typename T, typename S>
void run_rbgs(const LevelDev& L, int colour, S* z, const T* b, hipStream_t s) {
    if (L.split) {
        const int ny = L.core_hi[1] - L.core_lo[1] + 1, nz = L.core_hi[2] - L.core_lo[2] + 1;
        if (ny <= 0 || nz <= 0 || L.hx <= 0) return;
        if (L.hx % 4 || !L.lab_split) throw Error(IIM_E_INTERNAL, "colour-split rows must hold a multiple of 4");
        // four entries per thread: periodic rows must hold exactly n / 2 entries (their seam wrap)
        if (L.half >= SPLIT4_MIN_ENTRIES && (!L.periodic || 2 * L.hx == L.n)) {
            const int nq = L.hx / 4, nrows = ny * nz;
            const int64_t nthreads = (int64_t)nq * nrows;
            if (nthreads > INT32_MAX - 256) throw Error(IIM_E_INTERNAL, "level too large for the half-sweep grid");
            hipLaunchKernelGGL((k_rbgs_split<T, S>), dim3((unsigned)cdiv(nthreads, 256)), dim3(256), 0, s, L, colour,
                               nq, ny, nrows, z, b);
        } else {
            const int gx = cdiv(L.hx, 64), gy = cdiv(ny, 4);
            hipLaunchKernelGGL((k_rbgs_split1<T, S>), dim3(gx * gy * nz), dim3(256), 0, s, L, colour, gx, gy, z, b);
        }
        IIM_LAUNCH_CHECK();
        return;
    }
    dim3 g, k;
    level_grid(L, &g, &k);
    g.x = cdiv(cdiv(std::max(L.core_hi[0] - L.core_lo[0] + 1, 1), 2), 64);  // a thread per pair of nodes
    if (L.dim == 2)
        hipLaunchKernelGGL((k_rbgs<T, S, 2>), g, k, 0, s, L, colour, z, b);
    else
        hipLaunchKernelGGL((k_rbgs<T, S, 3>), g, k, 0, s, L, colour, z, b);
    IIM_LAUNCH_CHECK();
}

template <typename T, typename S>
void run_sw_apply(const LevelDev& L, const S* z, T* y, hipStream_t s) {
    dim3 g, k;
    level_grid(L, &g, &k);
    if (L.dim == 2)
        hipLaunchKernelGGL((k_sw_apply<T, S, 2>), g, k, 0, s, L, z, y);
    else
        hipLaunchKernelGGL((k_sw_apply<T, S, 3>), g, k, 0, s, L, z, y);
    IIM_LAUNCH_CHECK();
}

template <typename T, typename S>
void run_resid_restrict(const LevelDev& F, const LevelDev& C, const S* z, const T* b, T* bc, hipStream_t s, S* zc0) {
    if (zc0 && F.dim != 3) throw Error(IIM_E_INTERNAL, "coarse iterate start is built for 3D levels");
    dim3 g, k;
    level_grid(C, &g, &k);
    if (F.dim == 2)
        hipLaunchKernelGGL((k_resid_restrict<T, S, 2>), g, k, 0, s, F, C, z, b, bc);
    else
        hipLaunchKernelGGL((k_restrict3<T, S>), dim3(g.x * g.y * g.z), dim3(256), 0, s, F, C, (int)g.x, (int)g.y, z, b,
                           bc, zc0);
    IIM_LAUNCH_CHECK();
}

template <typename T, typename S>
void run_prolong(const LevelDev& F, const LevelDev& C, int mode, const S* zc, S* z, hipStream_t s) {
    if (F.dim == 3) {
        // coarse cells whose fine nodes meet the fine core
        int c0[3], nc[3];
        for (int d = 0; d < 3; ++d) {
            c0[d] = F.core_lo[d] >> 1;
            nc[d] = (F.core_hi[d] >> 1) - c0[d] + 1;
            if (F.core_hi[d] < F.core_lo[d]) return;
        }
        const int64_t ntot = (int64_t)nc[0] * nc[1] * nc[2];
        if (ntot > INT32_MAX - 256) throw Error(IIM_E_INTERNAL, "level too large for the prolongation grid");
        hipLaunchKernelGGL((k_prolong_cells<T, S>), dim3((unsigned)cdiv(ntot, 256)), dim3(256), 0, s, F, C, mode,
                           c0[0], c0[1], c0[2], nc[0], nc[1], (int)ntot, zc, z);
        IIM_LAUNCH_CHECK();
        return;
    }
    dim3 g, k;
    level_grid(F, &g, &k);
    hipLaunchKernelGGL((k_prolong<T, S, 2>), g, k, 0, s, F, C, mode, zc, z);
    IIM_LAUNCH_CHECK();
}

template <typename T, typename S>
void run_coarse_solve(const LevelDev& L, const int32_t* list, int64_t nc, const T* Ainv, const T* b, S* z,
                      hipStream_t s) {
    if (nc == 0) return;
    hipLaunchKernelGGL((k_coarse_solve<T, S>), dim3(cdiv(nc, 64)), dim3(64), 0, s, list, nc, Ainv, b, z);
    IIM_LAUNCH_CHECK();
}

template <typename S>
void run_zero(S* p, int64_t n, hipStream_t s) {
    if (n == 0) return;
    int blocks = (int)std::min<int64_t>(cdiv(n, 256), 4096);
    hipLaunchKernelGGL((k_zero<S>), dim3(blocks), dim3(256), 0, s, p, n);
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// precision boundary
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_cast_in(LevelDev L, const double* v, const double* scale, double h2, double bp, double bm, T* rhs) {
    int64_t n = L.box.size();
    double sc = *scale;
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < n; l += (int64_t)gridDim.x * blockDim.x) {
        uint8_t kk = L.labels[l] & KIND_MASK;
        double val = 0.0;
        if (kk == K_PLUS) val = sc * h2 * v[l] / bp;
        else if (kk == K_MINUS) val = sc * h2 * v[l] / bm;
        rhs[l] = (T)val;
    }
}

template <typename S>
__global__ void k_cast_out(LevelDev L, const S* z, const double* scale, double* out) {
    int64_t n = L.box.size();
    double inv = 1.0 / *scale;
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < n; l += (int64_t)gridDim.x * blockDim.x) {
        double val = is_unknown(L.labels[l]) ? (double)load_it<double, S>(z, l) * inv : 0.0;
        out[l] = val;
    }
}

// Colour-split level: a block covers 64 entries of two box rows in both
// colours (wavefront g: colour g & 1, row 2 * pair + (g >> 1)), so the
// box-order reads and writes of a row are shared by two wavefronts of a block.
struct SplitEntry {
    bool ok;     // entry inside the vector
    bool node;   // entry holds a node of the box
    int64_t l;   // box index of that node
    int64_t v;   // index in the level vector
};
__device__ inline SplitEntry split_entry(const LevelDev& L, int gxm) {
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int chunk = blockIdx.x % gxm, pair = blockIdx.x / gxm;
    const int m = chunk * 64 + lane, r = 2 * pair + (g >> 1), colour = g & 1;
    const int nrows = L.box.dims[1] * L.box.dims[2];
    SplitEntry e{false, false, 0, 0};
    if (m >= L.hx || r >= nrows) return e;
    const int j = L.box.lo[1] + r % L.box.dims[1], k = L.box.lo[2] + r / L.box.dims[1];
    const int a = 2 * m + ((colour ^ (L.box.lo[0] + j + k)) & 1);
    e.ok = true;
    e.node = a < L.box.dims[0];
    e.l = (int64_t)a + (int64_t)L.box.dims[0] * r;
    e.v = (int64_t)colour * L.half + (int64_t)r * L.hx + m;
    return e;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cast_in_split(LevelDev L, int gxm, const double* v, const double* scale,
                                                       double h2, double bp, double bm, T* rhs) {
    const SplitEntry e = split_entry(L, gxm);
    if (!e.ok) return;
    double val = 0.0;
    if (e.node) {
        const uint8_t kk = L.labels[e.l] & KIND_MASK;
        const double sc = *scale;
        if (kk == K_PLUS) val = sc * h2 * v[e.l] / bp;
        else if (kk == K_MINUS) val = sc * h2 * v[e.l] / bm;
    }
    rhs[e.v] = (T)val;
}

template <typename S>
__global__ void __launch_bounds__(256) k_cast_out_split(LevelDev L, int gxm, const S* z, const double* scale,
                                                        double* out) {
    const SplitEntry e = split_entry(L, gxm);
    if (!e.ok || !e.node) return;
    const double inv = 1.0 / *scale;
    out[e.l] = is_unknown(L.labels[e.l]) ? (double)load_it<double, S>(z, e.v) * inv : 0.0;
}

static inline int split_blocks(const LevelDev& L, int* gxm) {
    *gxm = cdiv(L.hx, 64);
    return *gxm * cdiv((int64_t)L.box.dims[1] * L.box.dims[2], 2);
}

template <typename T>
void run_cast_in(const LevelDev& L, const double* v, const double* scale_dev, double h2, double bp, double bm, T* rhs,
                 hipStream_t s) {
    if (L.split) {
        int gxm;
        const int nb = split_blocks(L, &gxm);
        hipLaunchKernelGGL((k_cast_in_split<T>), dim3(nb), dim3(256), 0, s, L, gxm, v, scale_dev, h2, bp, bm, rhs);
        IIM_LAUNCH_CHECK();
        return;
    }
    int blocks = (int)std::min<int64_t>(cdiv(L.box.size(), 256), 4096);
    hipLaunchKernelGGL((k_cast_in<T>), dim3(blocks), dim3(256), 0, s, L, v, scale_dev, h2, bp, bm, rhs);
    IIM_LAUNCH_CHECK();
}

template <typename S>
void run_cast_out(const LevelDev& L, const S* z, const double* scale_dev, double* out, hipStream_t s) {
    if (L.split) {
        int gxm;
        const int nb = split_blocks(L, &gxm);
        hipLaunchKernelGGL((k_cast_out_split<S>), dim3(nb), dim3(256), 0, s, L, gxm, z, scale_dev, out);
        IIM_LAUNCH_CHECK();
        return;
    }
    int blocks = (int)std::min<int64_t>(cdiv(L.box.size(), 256), 4096);
    hipLaunchKernelGGL((k_cast_out<S>), dim3(blocks), dim3(256), 0, s, L, z, scale_dev, out);
    IIM_LAUNCH_CHECK();
}

template <typename T, typename S>
void run_cast_sweep0(const LevelDev& L, const double* v, const double* scale_dev, double h2, double bp, double bm,
                     T* b, S* z, hipStream_t s) {
    if (!L.split || L.dim != 3) throw Error(IIM_E_INTERNAL, "cast + first half-sweep needs a colour-split 3D level");
    const int64_t nthreads = (int64_t)L.hx * L.box.dims[1] * L.box.dims[2];
    if (nthreads > INT32_MAX - 256) throw Error(IIM_E_INTERNAL, "level too large for the cast grid");
    hipLaunchKernelGGL((k_cast_sweep0<T, S>), dim3((unsigned)cdiv(nthreads, 256)), dim3(256), 0, s, L, v, scale_dev,
                       h2, bp, bm, b, z);
    IIM_LAUNCH_CHECK();
}

template <typename T, typename S>
void run_rbgs_out(const LevelDev& L, const S* z, const T* b, double* out, const double* scale_dev, hipStream_t s) {
    if (!L.split || L.dim != 3) throw Error(IIM_E_INTERNAL, "half-sweep with output needs a colour-split 3D level");
    const int ny = L.core_hi[1] - L.core_lo[1] + 1, nz = L.core_hi[2] - L.core_lo[2] + 1;
    if (ny <= 0 || nz <= 0 || L.hx <= 0) return;
    const int64_t nthreads = (int64_t)L.hx * ny * nz;
    if (nthreads > INT32_MAX - 256) throw Error(IIM_E_INTERNAL, "level too large for the half-sweep grid");
    hipLaunchKernelGGL((k_rbgs_split_out<T, S>), dim3((unsigned)cdiv(nthreads, 256)), dim3(256), 0, s, L, ny,
                       ny * nz, z, b, out, scale_dev);
    IIM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// storage box <-> level layout
// ---------------------------------------------------------------------------
template <typename U>
__global__ void k_box_level(LevelDev L, const U* src, U* dst, int to_level) {
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < L.box.size();
         l += (int64_t)gridDim.x * blockDim.x) {
        int ijk[3];
        L.box.coords(l, ijk);
        const int64_t v = vidx(L, ijk[0], ijk[1], ijk[2]);
        if (to_level) dst[v] = src[l];
        else dst[l] = src[v];
    }
}

template <typename U>
void run_box_to_level(const LevelDev& L, const U* boxed, U* lev, hipStream_t s) {
    if (L.split) IIM_HIP(hipMemsetAsync(lev, 0, vsize(L) * sizeof(U), s));  // entries of no node stay zero
    const int blocks = (int)std::min<int64_t>(cdiv(L.box.size(), 256), 4096);
    hipLaunchKernelGGL((k_box_level<U>), dim3(blocks), dim3(256), 0, s, L, boxed, lev, 1);
    IIM_LAUNCH_CHECK();
}

template <typename U>
void run_level_to_box(const LevelDev& L, const U* lev, U* boxed, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(cdiv(L.box.size(), 256), 4096);
    hipLaunchKernelGGL((k_box_level<U>), dim3(blocks), dim3(256), 0, s, L, lev, boxed, 0);
    IIM_LAUNCH_CHECK();
}
template void run_box_to_level<uint8_t>(const LevelDev&, const uint8_t*, uint8_t*, hipStream_t);
template void run_box_to_level<double>(const LevelDev&, const double*, double*, hipStream_t);
template void run_box_to_level<float>(const LevelDev&, const float*, float*, hipStream_t);
template void run_box_to_level<__half>(const LevelDev&, const __half*, __half*, hipStream_t);
template void run_level_to_box<double>(const LevelDev&, const double*, double*, hipStream_t);
template void run_level_to_box<float>(const LevelDev&, const float*, float*, hipStream_t);
template void run_level_to_box<__half>(const LevelDev&, const __half*, __half*, hipStream_t);

// ---------------------------------------------------------------------------
// full grid <-> storage box
// ---------------------------------------------------------------------------
__global__ void k_full_to_box(int dim, int n, Box b, const double* full, double* boxed, const uint8_t* labels,
                              int only_unknowns) {
    int64_t tot = b.size();
    int64_t n1 = n + 1;
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < tot; l += (int64_t)gridDim.x * blockDim.x) {
        int ijk[3];
        b.coords(l, ijk);
        bool in = true;
        for (int d = 0; d < dim; ++d) in = in && ijk[d] >= 0 && ijk[d] <= n;
        double v = 0.0;
        if (in) {
            uint8_t kk = labels[l] & KIND_MASK;
            bool take = only_unknowns == 1 ? (kk == K_PLUS || kk == K_MINUS) : (only_unknowns == 2 ? kk == K_BOX : true);
            if (take) v = full[ijk[0] + n1 * (ijk[1] + n1 * (int64_t)ijk[2])];
        }
        boxed[l] = v;
    }
}

void run_full_to_box(int dim, int n, const Box& b, const double* full, double* boxed, const uint8_t* labels,
                     int only_unknowns, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(cdiv(b.size(), 256), 8192);
    hipLaunchKernelGGL(k_full_to_box, dim3(blocks), dim3(256), 0, s, dim, n, b, full, boxed, labels, only_unknowns);
    IIM_LAUNCH_CHECK();
}

__global__ void k_box_to_full(int dim, int n, Box b, const double* boxed, const uint8_t* labels, double fill,
                              double* full) {
    int64_t n1 = n + 1;
    int64_t tot = dim == 2 ? n1 * n1 : n1 * n1 * n1;
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < tot; f += (int64_t)gridDim.x * blockDim.x) {
        int ijk[3] = {(int)(f % n1), (int)((f / n1) % n1), dim == 3 ? (int)(f / (n1 * n1)) : 0};
        bool inb = true;
        for (int d = 0; d < 3; ++d) inb = inb && ijk[d] >= b.lo[d] && ijk[d] < b.lo[d] + b.dims[d];
        double v = fill;
        if (inb) {
            int64_t l = b.idx(ijk[0], ijk[1], ijk[2]);
            if (is_unknown(labels[l])) v = boxed[l];
        }
        full[f] = v;
    }
}

void run_box_to_full(int dim, int n, const Box& b, const double* boxed, const uint8_t* labels, double fill,
                     double* full, hipStream_t s) {
    int64_t n1 = n + 1;
    int64_t tot = dim == 2 ? n1 * n1 : n1 * n1 * n1;
    int blocks = (int)std::min<int64_t>(cdiv(tot, 256), 8192);
    hipLaunchKernelGGL(k_box_to_full, dim3(blocks), dim3(256), 0, s, dim, n, b, boxed, labels, fill, full);
    IIM_LAUNCH_CHECK();
}

// explicit instantiations
#define INST_TS(T, S)                                                                                     \
    template void run_rbgs<T, S>(const LevelDev&, int, S*, const T*, hipStream_t);                        \
    template void run_resid_restrict<T, S>(const LevelDev&, const LevelDev&, const S*, const T*, T*,      \
                                           hipStream_t, S*);                                              \
    template void run_prolong<T, S>(const LevelDev&, const LevelDev&, int, const S*, S*, hipStream_t);    \
    template void run_sw_apply<T, S>(const LevelDev&, const S*, T*, hipStream_t);                         \
    template void run_cast_sweep0<T, S>(const LevelDev&, const double*, const double*, double, double, double, T*, \
                                        S*, hipStream_t);                                                             \
    template void run_rbgs_out<T, S>(const LevelDev&, const S*, const T*, double*, const double*, hipStream_t);     \
    template void run_coarse_solve<T, S>(const LevelDev&, const int32_t*, int64_t, const T*, const T*, S*, \
                                         hipStream_t);                                                    \
    template void run_tail<T, S>(int, const TailDev*, int64_t, hipStream_t);                              \
    template void run_tail_batch<T, S>(int, const TailBatch&, hipStream_t);                               \
    template bool run_down_fused<T, S>(const LevelDev&, const LevelDev&, const T*, S*, T*, int, hipStream_t,      \
                                       const CastInArgs*);                                                           \
    template bool run_up_fused<T, S>(const LevelDev&, const LevelDev&, int, const S*, const T*, const S*, S*, int, \
                                     hipStream_t, double*, const double*);
INST_TS(double, double)
INST_TS(float, float)
INST_TS(float, __half)
template void run_zero<double>(double*, int64_t, hipStream_t);
template void run_zero<float>(float*, int64_t, hipStream_t);
template void run_zero<__half>(__half*, int64_t, hipStream_t);
template void run_cast_in<double>(const LevelDev&, const double*, const double*, double, double, double, double*,
                                  hipStream_t);
template void run_cast_in<float>(const LevelDev&, const double*, const double*, double, double, double, float*,
                                 hipStream_t);
template void run_cast_out<double>(const LevelDev&, const double*, const double*, double*, hipStream_t);
template void run_cast_out<float>(const LevelDev&, const float*, const double*, double*, hipStream_t);
template void run_cast_out<__half>(const LevelDev&, const __half*, const double*, double*, hipStream_t);

}  // namespace iim

namespace iim {

// Neumann apply weights: W_j = S_j - (Sc_j / Sc_n) S_n, data coefficient Sc_j / (beta Sc_n).
// One wave per control-point side, lanes over its entries (contiguous in every row).
__global__ void __launch_bounds__(256) k_combine_neumann(const int64_t* ptr, int64_t ncs, int w, int nrows,
                                                         const double* S, const double* Sc, double beta, int64_t nnz,
                                                         double* W, double* dcoef) {
    const int lane = threadIdx.x % 64;
    const int64_t cs = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64;
    if (cs >= ncs) return;
    const double scn = Sc[cs * nrows + w];
    const int64_t a0 = ptr[cs], a1 = ptr[cs + 1];
    for (int j = 0; j < w; ++j) {
        const double scj = Sc[cs * nrows + j];
        const double f = scj / scn;
        for (int64_t a = a0 + lane; a < a1; a += 64) W[j * nnz + a] = S[j * nnz + a] - f * S[w * nnz + a];
        if (lane == 0) dcoef[cs * w + j] = scj / (beta * scn);
    }
}

__global__ void k_copy_dcoef(int64_t ncs, int w, int nrows, const double* Sc, double* dcoef) {
    int64_t cs = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (cs >= ncs) return;
    for (int j = 0; j < w; ++j) dcoef[cs * w + j] = Sc[cs * nrows + j];
}

void run_apply_weights(int bc, const int64_t* ptr, int64_t ncs, int w, int nrows, const double* S, const double* Sc,
                       double beta, int64_t nnz, double* W, double* dcoef, hipStream_t s) {
    if (ncs == 0) return;
    if (bc == IIM_BC_NEUMANN)
        hipLaunchKernelGGL(k_combine_neumann, dim3(cdiv(ncs * 64, 256)), dim3(256), 0, s, ptr, ncs, w, nrows, S, Sc,
                           beta, nnz, W, dcoef);
    else
        hipLaunchKernelGGL(k_copy_dcoef, dim3(cdiv(ncs, 128)), dim3(128), 0, s, ncs, w, nrows, Sc, dcoef);
    IIM_LAUNCH_CHECK();
}

__device__ inline double to_d(double v) { return v; }
__device__ inline double to_d(float v) { return (double)v; }
__device__ inline double to_d(__half v) { return (double)__half2float(v); }
__device__ inline void from_d(double v, double* p) { *p = v; }
__device__ inline void from_d(double v, float* p) { *p = (float)v; }
__device__ inline void from_d(double v, __half* p) { *p = __float2half((float)v); }

template <typename A, typename B>
__global__ void k_convert(const A* a, B* b, int64_t n, double scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        from_d(to_d(a[i]) * scale, &b[i]);
}

template <typename A, typename B>
void run_convert(const A* a, B* b, int64_t n, double scale, hipStream_t s) {
    if (n == 0) return;
    int blocks = (int)std::min<int64_t>(cdiv(n, 256), 4096);
    hipLaunchKernelGGL((k_convert<A, B>), dim3(blocks), dim3(256), 0, s, a, b, n, scale);
    IIM_LAUNCH_CHECK();
}
template void run_convert<double, double>(const double*, double*, int64_t, double, hipStream_t);
template void run_convert<double, float>(const double*, float*, int64_t, double, hipStream_t);
template void run_convert<double, __half>(const double*, __half*, int64_t, double, hipStream_t);
template void run_convert<float, double>(const float*, double*, int64_t, double, hipStream_t);
template void run_convert<__half, double>(const __half*, double*, int64_t, double, hipStream_t);

}  // namespace iim
