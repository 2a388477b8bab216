// Least-squares ghost stencils, one wavefront per control point and side
// (Sec. 2.1-2.2 of the paper).
//
// The interpolation set holds x_c, then the side's unknowns inside the
// half-ellipse (2D) / half-ellipsoid (3D) with tangential semi-axis a and
// normal semi-axis b (units of h), in increasing flat order, minus the one
// closest to x_c.  The monomials of total degree <= k-1 in xi = (y - x_c)/(a h)
// form A; one Householder QR A = QR gives every stencil as s = Q R^{-T} e
// (one triangular solve and one product with Q per stencil).
//
// Wave layout: candidates of the search window are visited 64 at a time in
// increasing flat order and compacted with a ballot, so the set order is the
// flat order regardless of timing; the QR keeps A column-major in a per-wave
// global scratch slab (lanes own rows); every reduction has a fixed order
// (VALU DPP reductions in the register QR, xor butterflies elsewhere), so
// results do not depend on scheduling.
#include "kernels.h"

namespace iim {

// On a periodic grid a node index i (0..n-1) is taken at the image nearest to
// the control point coordinate xcd (a fit spans a few h, the cell n h): the
// unwrapped index, whose coordinate lo + i h is then formed as for any node.
__device__ inline int unwrap_near(const Geom& g, int i, double xcd) {
    if (!g.periodic) return i;
    const double t = (xcd - g.lo) / g.h - (double)i;
    return i + g.n * (int)llround(t / (double)g.n);
}


constexpr int LS_MAXC = 1024;  // candidates kept per set (LDS list)
constexpr int LS_RROWS = 12;   // rows per lane of a register-held column (768 = the 3D slab height)
constexpr double SET_TOL = 1e-12;
constexpr double RANK_TOL = 1e-10;

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// monomial exponents of total degree <= deg: 2D (i, t-i) i = t..0; 3D (i, j, t-i-j)
__device__ inline int monomials(int dim, int deg, int (*e)[3]) {
    int c = 0;
    for (int t = 0; t <= deg; ++t) {
        if (dim == 2) {
            for (int i = t; i >= 0; --i) {
                e[c][0] = i;
                e[c][1] = t - i;
                e[c][2] = 0;
                ++c;
            }
        } else {
            for (int i = t; i >= 0; --i)
                for (int j = t - i; j >= 0; --j) {
                    e[c][0] = i;
                    e[c][1] = j;
                    e[c][2] = t - i - j;
                    ++c;
                }
        }
    }
    return c;
}

__device__ inline double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// Householder QR of the (M x PT) least-squares matrix held in registers: lane l
// owns rows l, l + 64, ... (RPL rows).  Column indices are compile-time after
// unrolling, so A never leaves the register file.  Returns false if the rank
// test fails.  With want_weights, writes the stencils s = Q R^{-T} e for the
// functionals in E (nrows <= 4) to S_out / Sc_out exactly like the scratch path.
// (inlined: as a called function it kept A's spill slots in scratch memory)
template <int PT, int RPL>
__device__ __attribute__((always_inline)) bool reg_qr(int M, int lane, int dim, const int32_t* list_idx, int closest,
                                                      const Box& b, const Geom& g, const double* xc, double sc,
                                                      const int (*ex)[3], bool want_weights, int nrows,
                                                      const double (*E)[84], double (*Y)[4], double* tauv,
                                                      double (*Rs)[PT], int64_t base, int64_t nnz, int64_t cs,
                                                      int32_t* idx_out, double* S_out, double* Sc_out) {
    double A[RPL][PT];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        double xi[3] = {0.0, 0.0, 0.0};
        const bool live = r < M;
        if (live && r > 0) {
            int li = list_idx[r - 1 + (r - 1 >= closest ? 1 : 0)];
            int ijk[3];
            b.coords(li, ijk);
            for (int d = 0; d < dim; ++d) xi[d] = (node_coord(g, unwrap_near(g, ijk[d], xc[d])) - xc[d]) / sc;
        }
#pragma unroll
        for (int c = 0; c < PT; ++c)
            A[q][c] = live ? ipow(xi[0], ex[c][0]) * ipow(xi[1], ex[c][1]) * ipow(xi[2], ex[c][2]) : 0.0;
    }
    double rmax = 0.0, rmin = 1e300;
#pragma unroll
    for (int c = 0; c < PT; ++c) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < RPL; ++q)
            if (lane + 64 * q > c) s += A[q][c] * A[q][c];
        s = wave_sum_valu(s);
        const double alpha = lane_value(A[0][c], c);
        const double norm = sqrt(alpha * alpha + s);
        double tau = 0.0, beta = alpha;
        if (s != 0.0) {
            beta = alpha >= 0.0 ? -norm : norm;
            tau = (beta - alpha) / beta;
            const double inv = 1.0 / (alpha - beta);
#pragma unroll
            for (int q = 0; q < RPL; ++q)
                if (lane + 64 * q > c) A[q][c] *= inv;
        }
        if (lane == 0) tauv[c] = tau;
        rmax = fmax(rmax, fabs(beta));
        rmin = fmin(rmin, fabs(beta));
        // dots with every trailing column, reduced together in chunks of 8
#pragma unroll
        for (int c0 = c + 1; c0 < PT; c0 += 8) {
            double d[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                d[t] = 0.0;
                if (c0 + t < PT) {
#pragma unroll
                    for (int q = 0; q < RPL; ++q)
                        if (lane + 64 * q > c) d[t] += A[q][c] * A[q][c0 + t];
                }
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (c0 + t < PT) d[t] = wave_sum_valu(d[t]) + lane_value(A[0][c0 + t], c);
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (c0 + t < PT) {
                    const double f = tau * d[t];
#pragma unroll
                    for (int q = 0; q < RPL; ++q)
                        if (lane + 64 * q > c) A[q][c0 + t] -= f * A[q][c];
                    if (lane == c) A[0][c0 + t] -= f;
                }
        }
        if (lane == c) A[0][c] = beta;
    }
    if (rmin < RANK_TOL * rmax) return false;
    if (!want_weights) return true;
    // R (upper triangle, row i held by lane i) to LDS
#pragma unroll
    for (int c = 0; c < PT; ++c)
        if (lane < PT && lane <= c) Rs[lane][c] = A[0][c];
    __syncthreads();
    // R^T Y = E^T by columns: lane j keeps E_j minus the terms known so far and
    // subtracts R_ij y_i as soon as y_i is known (the same operations, in the same
    // order, as the row-by-row substitution)
    {
        double acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = (k < nrows && lane < PT) ? E[k][lane] : 0.0;
#pragma unroll 1
        for (int i = 0; i < PT; ++i) {
            const double rii = Rs[i][i];
            const double rij = (lane > i && lane < PT) ? Rs[i][lane] : 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k >= nrows) break;
                const double yi = lane_value(acc[k], i) / rii;
                if (lane == 0) Y[i][k] = yi;
                if (lane > i) acc[k] -= rij * yi;
            }
        }
    }
    __syncthreads();
    double sv[4][RPL];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int r = lane + 64 * q;
            sv[k][q] = (k < nrows && r < PT) ? Y[r][k] : 0.0;
        }
    // s = Q [Y; 0]: reflectors in reverse order
#pragma unroll
    for (int c = PT - 1; c >= 0; --c) {
        const double tau = tauv[c];
        double d[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            d[k] = 0.0;
#pragma unroll
            for (int q = 0; q < RPL; ++q)
                if (lane + 64 * q > c) d[k] += A[q][c] * sv[k][q];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nrows) d[k] = wave_sum_valu(d[k]) + lane_value(sv[k][0], c);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nrows) {
                const double f = tau * d[k];
#pragma unroll
                for (int q = 0; q < RPL; ++q)
                    if (lane + 64 * q > c) sv[k][q] -= f * A[q][c];
                if (lane == c) sv[k][0] -= f;
            }
    }
    if (lane == 0)
        for (int k = 0; k < nrows; ++k) Sc_out[cs * nrows + k] = sv[k][0];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        if (r >= 1 && r < M) {
            int li = list_idx[r - 1 + (r - 1 >= closest ? 1 : 0)];
            if (idx_out) idx_out[base + r - 1] = li;
            for (int k = 0; k < nrows; ++k) S_out[(int64_t)k * nnz + base + r - 1] = sv[k][q];
        }
    }
    return true;
}

template <int PT, int RPL>
__global__ void __launch_bounds__(64) k_ls(Geom g, Box b, const uint8_t* labels, CPDev cp, LSParams P, int pass,
                                           int32_t* m_out, int32_t* grow_out, const int64_t* ptr, int32_t* idx_out,
                                           double* S_out, double* Sc_out, double* scratch, int* err,
                                           const int32_t* cs_list, int64_t n_list, uint8_t* route) {
    __shared__ int32_t list_idx[LS_MAXC];
    __shared__ double list_r2[LS_MAXC];
    __shared__ int ex[84][3];
    __shared__ double tauv[84];
    __shared__ double Y[84][4];
    __shared__ double E[4][84];
    __shared__ double Rs[PT][PT];
    const int lane = threadIdx.x;
    const int K = P.order_k;
    const int p = g.dim == 2 ? K * (K + 1) / 2 : K * (K + 1) * (K + 2) / 6;
    if (lane == 0) monomials(g.dim, K - 1, ex);
    __syncthreads();
    const int64_t ncs = cp.ncp * P.nsides;
    const int mcap = P.mcap;
    // per-wave slab of the scratch launch: [p][mcap] columns of A, then s [4][mcap]
    double* Acol = scratch ? scratch + (int64_t)blockIdx.x * (int64_t)(p + 4) * mcap : nullptr;
    double* Scol = scratch ? Acol + (int64_t)p * mcap : nullptr;

    // cs_list == nullptr: every fit through the register path, fits larger than it
    // are routed (route[cs] = 1) to a second launch over cs_list with scratch
    const int64_t nwork = cs_list ? n_list : ncs;
    for (int64_t wk = blockIdx.x; wk < nwork; wk += gridDim.x) {
        const int64_t cs = cs_list ? cs_list[wk] : wk;
        if (!cs_list && pass == 1 && route[cs]) continue;
        const int64_t c = cs / P.nsides;
        const int sidx = (int)(cs % P.nsides);
        const uint8_t side = sidx == 0 ? K_PLUS : K_MINUS;
        double xc[3], nrm[3], nu[3];
        for (int d = 0; d < 3; ++d) {
            xc[d] = cp.x[d * cp.ncp + c];
            nrm[d] = cp.n[d * cp.ncp + c];
            nu[d] = sidx == 0 ? nrm[d] : -nrm[d];
        }
        const int axis = cp.axis[c];
        const int64_t anode = cp.a[sidx * cp.ncp + c];
        const int adir = cp.dir[sidx * cp.ncp + c];
        int g0 = 0, g1 = P.max_grow;
        if (pass == 1) {
            g0 = g1 = grow_out[cs];
            if (g0 < 0) continue;
        }
        bool done = false;
        for (int grow = g0; grow <= g1 && !done; ++grow) {
            const double a = P.a0 + 0.5 * grow, bb = P.b0 + 0.5 * grow;
            const int R = (int)ceil(fmax(a, bb)) + 1;
            int wlo[3] = {0, 0, 0}, wlen[3] = {1, 1, 1};
            for (int d = 0; d < g.dim; ++d) {
                int ci = (int)floor((xc[d] - g.lo) / g.h + 0.5);
                // periodic: the window is unwrapped (no clamp); labels and indices wrap below
                int lo = g.periodic ? ci - R : max(0, ci - R), hi = g.periodic ? ci + R : min(g.n, ci + R);
                wlo[d] = lo;
                wlen[d] = hi - lo + 1;
            }
            const int total = wlen[0] * wlen[1] * wlen[2];
            int count = 0;
            bool overflow = false;
            for (int base = 0; base < total; base += 64) {
                int t = base + lane;
                bool keep = false;
                int32_t lidx = 0;
                double r2 = 0.0;
                if (t < total) {
                    int ijk[3] = {wlo[0] + t % wlen[0], wlo[1] + (t / wlen[0]) % wlen[1], wlo[2] + t / (wlen[0] * wlen[1])};
                    int wk3[3] = {ijk[0], ijk[1], ijk[2]};
                    if (g.periodic)
                        for (int d = 0; d < g.dim; ++d) wk3[d] = wrap_index(ijk[d], g.n);
                    bool inbox = true;
                    for (int d = 0; d < 3; ++d) inbox = inbox && wk3[d] >= b.lo[d] && wk3[d] < b.lo[d] + b.dims[d];
                    if (inbox) {
                        lidx = (int32_t)b.idx(wk3[0], wk3[1], wk3[2]);
                        if ((labels[lidx] & KIND_MASK) == side) {
#pragma clang fp contract(off)
                            double nn = 0.0;
                            for (int d = 0; d < g.dim; ++d) {
                                double delta = (node_coord(g, ijk[d]) - xc[d]) / g.h;
                                nn += delta * nu[d];
                                r2 += delta * delta;
                            }
                            double t2 = fmax(r2 - nn * nn, 0.0);
                            keep = (nn >= -SET_TOL) && (t2 / (a * a) + nn * nn / (bb * bb) <= 1.0 + SET_TOL);
                        }
                    }
                }
                unsigned long long mask = __ballot(keep);
                int before = __popcll(mask & ((1ull << lane) - 1ull));
                if (keep) {
                    int pos = count + before;
                    if (pos < LS_MAXC) {
                        list_idx[pos] = lidx;
                        list_r2[pos] = r2;
                    }
                }
                count += __popcll(mask);
                if (count > LS_MAXC) overflow = true;
            }
            __syncthreads();
            if (overflow) {
                if (lane == 0) atomicOr(err, 32);
                break;
            }
            if (count == 0) continue;  // no candidates: grow
            // closest candidate: minimal r2, ties within SET_TOL to the lowest index (first in list)
            double dmin = 1e300;
            for (int i = lane; i < count; i += 64) dmin = fmin(dmin, list_r2[i]);
            dmin = wave_min(dmin);
            int closest = count;
            for (int i = lane; i < count; i += 64)
                if (list_r2[i] <= dmin + SET_TOL) closest = min(closest, i);
            for (int off = 32; off > 0; off >>= 1) closest = min(closest, __shfl_xor(closest, off, 64));
            const int m = count - 1;
            const int M = m + 1;  // rows: x_c then the m points
            if (M < p) continue;  // too few points: grow
            const double sc = a * g.h;
            if (M <= 64 * RPL && p == PT) {
                // register-resident QR (the common case)
                const bool stage = pass == 0 && idx_out != nullptr;
                if (pass == 1 && ptr[cs + 1] - ptr[cs] != m) {
                    if (lane == 0) atomicOr(err, 256);
                    break;
                }
                if (pass == 1 || stage) {
                    // evaluation functionals
                    int acoord[3];
                    b.coords(anode, acoord);
                    double xa[3] = {0.0, 0.0, 0.0};
                    for (int d = 0; d < g.dim; ++d) xa[d] = node_coord(g, unwrap_near(g, acoord[d], xc[d]));
                    for (int k = 0; k < P.nrows; ++k)
                        for (int col = lane; col < p; col += 64) {
                            double val;
                            if (k < P.w) {
                                double xg[3] = {xa[0], xa[1], xa[2]};
                                xg[axis] = xa[axis] + (double)((k + 1) * adir) * g.h;
                                double xi[3] = {0.0, 0.0, 0.0};
                                for (int d = 0; d < g.dim; ++d) xi[d] = (xg[d] - xc[d]) / sc;
                                val = ipow(xi[0], ex[col][0]) * ipow(xi[1], ex[col][1]) * ipow(xi[2], ex[col][2]);
                            } else {
                                // row w: d/dn; rows w + 1 + d: d/dx_d (gradient fits)
                                int deg = ex[col][0] + ex[col][1] + ex[col][2];
                                val = 0.0;
                                if (deg == 1) {
                                    int d = ex[col][0] ? 0 : (ex[col][1] ? 1 : 2);
                                    const int r = k - P.w;
                                    val = (r == 0 ? nrm[d] : (d == r - 1 ? 1.0 : 0.0)) / sc;
                                }
                            }
                            E[k][col] = val;
                        }
                    __syncthreads();
                }
                // pass 1 writes into the CSR arrays; pass 0 with idx_out set writes into a
                // staging layout with a fixed segment of 64 * RPL entries per fit
                const int64_t seg = 64 * RPL;
                bool ok = reg_qr<PT, RPL>(M, lane, g.dim, list_idx, closest, b, g, xc, sc, ex, pass == 1 || stage,
                                          P.nrows, E, Y, tauv, Rs, pass == 1 ? ptr[cs] : cs * seg,
                                          pass == 1 ? ptr[ncs] : ncs * seg, cs, idx_out, S_out, Sc_out);
                __syncthreads();
                if (!ok) continue;  // rank deficient: grow
                done = true;
                if (pass == 0 && lane == 0) {
                    m_out[cs] = m;
                    grow_out[cs] = grow;
                }
                break;
            }
            if (!cs_list) {  // too large for registers: leave it to the scratch launch
                if (pass == 0 && lane == 0) {
                    route[cs] = 1;
                    grow_out[cs] = -3;
                    m_out[cs] = 0;
                }
                done = true;
                break;
            }
            if (M > mcap) {
                if (lane == 0) atomicOr(err, 32);
                break;
            }
            // assemble A (column-major), row 0 = x_c
            for (int r = lane; r < M; r += 64) {
                double xi[3] = {0.0, 0.0, 0.0};
                if (r > 0) {
                    int li = list_idx[r - 1 + (r - 1 >= closest ? 1 : 0)];
                    int ijk[3];
                    b.coords(li, ijk);
                    for (int d = 0; d < g.dim; ++d) xi[d] = (node_coord(g, unwrap_near(g, ijk[d], xc[d])) - xc[d]) / sc;
                }
                for (int col = 0; col < p; ++col)
                    Acol[(int64_t)col * mcap + r] = ipow(xi[0], ex[col][0]) * ipow(xi[1], ex[col][1]) *
                                                   ipow(xi[2], ex[col][2]);
            }
            __syncthreads();
            // Householder QR in panels of QP columns.  A panel is factored
            // column by column in the slab; its reflectors are then applied
            // to every later column held in registers (rows r = lane + 64 i),
            // one load and one store per column and panel instead of one per
            // reflector.  Each dot product is summed per lane over the same
            // rows in the same order as a column-at-a-time sweep whose lane L
            // takes rows col + 1 + L + 64 k, and its partials are moved to
            // those lanes before the wavefront sum, so the factors are the
            // same bit for bit.
            double rmax = 0.0, rmin = 1e300;
            constexpr int QP = 4;
            for (int c0 = 0; c0 < p; c0 += QP) {
                const int pe = min(c0 + QP, p);
                for (int col = c0; col < pe; ++col) {
                    double* v = Acol + (int64_t)col * mcap;
                    double s = 0.0;
                    for (int r = col + 1 + lane; r < M; r += 64) s += v[r] * v[r];
                    s = wave_sum(s);
                    double alpha = v[col];
                    double norm = sqrt(alpha * alpha + s);
                    double tau = 0.0, beta = alpha;
                    if (s != 0.0) {
                        beta = alpha >= 0.0 ? -norm : norm;
                        tau = (beta - alpha) / beta;
                        double inv = 1.0 / (alpha - beta);
                        for (int r = col + 1 + lane; r < M; r += 64) v[r] *= inv;
                    }
                    __syncthreads();
                    if (lane == 0) {
                        v[col] = beta;
                        tauv[col] = tau;
                    }
                    rmax = fmax(rmax, fabs(beta));
                    rmin = fmin(rmin, fabs(beta));
                    for (int c2 = col + 1; c2 < pe; ++c2) {  // the rest of the panel
                        double* u = Acol + (int64_t)c2 * mcap;
                        double dot = 0.0;
                        for (int r = col + 1 + lane; r < M; r += 64) dot += v[r] * u[r];
                        dot = wave_sum(dot) + u[col];
                        double f = tau * dot;
                        __syncthreads();
                        if (lane == 0) u[col] -= f;
                        for (int r = col + 1 + lane; r < M; r += 64) u[r] -= f * v[r];
                    }
                    __syncthreads();
                }
                if (pe >= p) break;
                double vv[QP][LS_RROWS];
#pragma unroll
                for (int t = 0; t < QP; ++t)
#pragma unroll
                    for (int i = 0; i < LS_RROWS; ++i) {
                        const int r = lane + 64 * i;
                        vv[t][i] = (c0 + t < pe && r < M) ? Acol[(int64_t)(c0 + t) * mcap + r] : 0.0;
                    }
                for (int c2 = pe; c2 < p; ++c2) {
                    double* u = Acol + (int64_t)c2 * mcap;
                    double uu[LS_RROWS];
#pragma unroll
                    for (int i = 0; i < LS_RROWS; ++i) {
                        const int r = lane + 64 * i;
                        uu[i] = r < M ? u[r] : 0.0;
                    }
#pragma unroll
                    for (int t = 0; t < QP; ++t) {
                        const int col = c0 + t;
                        if (col >= pe) break;
                        double part = 0.0;
#pragma unroll
                        for (int i = 0; i < LS_RROWS; ++i) {
                            const int r = lane + 64 * i;
                            if (r > col && r < M) part += vv[t][i] * uu[i];
                        }
                        // lane L of the column sweep summed rows col + 1 + L + 64 k
                        part = __shfl(part, (lane + col + 1) & 63, 64);
                        double ucol = 0.0;
#pragma unroll
                        for (int i = 0; i < LS_RROWS; ++i)
                            if (i == (col >> 6)) ucol = uu[i];
                        ucol = __shfl(ucol, col & 63, 64);
                        const double f = tauv[col] * (wave_sum(part) + ucol);
#pragma unroll
                        for (int i = 0; i < LS_RROWS; ++i) {
                            const int r = lane + 64 * i;
                            if (r == col) uu[i] -= f;
                            else if (r > col && r < M) uu[i] -= f * vv[t][i];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < LS_RROWS; ++i) {
                        const int r = lane + 64 * i;
                        if (r < M) u[r] = uu[i];
                    }
                }
                __syncthreads();
            }
            if (rmin < RANK_TOL * rmax) continue;  // rank deficient: grow
            done = true;
            if (pass == 0) {
                if (lane == 0) {
                    m_out[cs] = m;
                    grow_out[cs] = grow;
                }
                break;
            }
            // evaluation functionals: ghosts j = 1..w at anode + j adir e_axis, then d/dn
            int acoord[3];
            b.coords(anode, acoord);
            double xa[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < g.dim; ++d) xa[d] = node_coord(g, unwrap_near(g, acoord[d], xc[d]));
            for (int k = 0; k < P.nrows; ++k)
                for (int col = lane; col < p; col += 64) {
                    double val;
                    if (k < P.w) {
                        double xg[3] = {xa[0], xa[1], xa[2]};
                        xg[axis] = xa[axis] + (double)((k + 1) * adir) * g.h;
                        double xi[3] = {0.0, 0.0, 0.0};
                        for (int d = 0; d < g.dim; ++d) xi[d] = (xg[d] - xc[d]) / sc;
                        val = ipow(xi[0], ex[col][0]) * ipow(xi[1], ex[col][1]) * ipow(xi[2], ex[col][2]);
                    } else {
                        // row w: d/dn; rows w + 1 + d: d/dx_d (gradient fits)
                        int deg = ex[col][0] + ex[col][1] + ex[col][2];
                        val = 0.0;
                        if (deg == 1) {
                            int d = ex[col][0] ? 0 : (ex[col][1] ? 1 : 2);
                            const int r = k - P.w;
                            val = (r == 0 ? nrm[d] : (d == r - 1 ? 1.0 : 0.0)) / sc;
                        }
                    }
                    E[k][col] = val;
                }
            __syncthreads();
            // R^T Y = E^T (forward substitution), one lane per functional
            if (lane < P.nrows) {
                for (int i = 0; i < p; ++i) {
                    double acc = E[lane][i];
                    for (int l2 = 0; l2 < i; ++l2) acc -= Acol[(int64_t)i * mcap + l2] * Y[l2][lane];
                    Y[i][lane] = acc / Acol[(int64_t)i * mcap + i];
                }
            }
            __syncthreads();
            // s = Q [Y; 0]: apply the reflectors in reverse order
            for (int k = 0; k < P.nrows; ++k)
                for (int r = lane; r < M; r += 64) Scol[(int64_t)k * mcap + r] = r < p ? Y[r][k] : 0.0;
            __syncthreads();
            for (int col = p - 1; col >= 0; --col) {
                const double* v = Acol + (int64_t)col * mcap;
                double tau = tauv[col];
                double dots[4] = {0.0, 0.0, 0.0, 0.0};
                for (int k = 0; k < P.nrows; ++k) {
                    const double* s = Scol + (int64_t)k * mcap;
                    double d0 = 0.0;
                    for (int r = col + 1 + lane; r < M; r += 64) d0 += v[r] * s[r];
                    dots[k] = wave_sum(d0) + s[col];
                }
                __syncthreads();
                for (int k = 0; k < P.nrows; ++k) {
                    double* s = Scol + (int64_t)k * mcap;
                    double f = tau * dots[k];
                    if (lane == 0) s[col] -= f;
                    for (int r = col + 1 + lane; r < M; r += 64) s[r] -= f * v[r];
                }
                __syncthreads();
            }
            // write: Sc[cs][k] (weight of u(x_c)), S[k][ptr + alpha], idx
            const int64_t base = ptr[cs];
            const int64_t nnz = ptr[ncs];
            if (ptr[cs + 1] - base != m) {  // both passes enumerate the same set
                if (lane == 0) atomicOr(err, 256);
                break;
            }
            if (lane < P.nrows) Sc_out[cs * P.nrows + lane] = Scol[(int64_t)lane * mcap];
            for (int r = 1 + lane; r < M; r += 64) {
                int li = list_idx[r - 1 + (r - 1 >= closest ? 1 : 0)];
                idx_out[base + r - 1] = li;
                for (int k = 0; k < P.nrows; ++k) S_out[(int64_t)k * nnz + base + r - 1] = Scol[(int64_t)k * mcap + r];
            }
            __syncthreads();
        }
        if (!done && pass == 0 && lane == 0) {
            m_out[cs] = 0;
            grow_out[cs] = -1;
            atomicOr(err, 128);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3D fits of the (4,5) scheme (about 235 points, 35 monomials).  The candidate
// search, a chain of dependent label loads, runs in a kernel of its own with
// few registers and many waves per SIMD.
//
// k_ls3_search (one wavefront per fit) finds the smallest growth whose set has
// at least 35 points and writes the set, without its point closest to x_c,
// into the fit's staging segment.  Sets larger than 256 points are routed to
// the global-memory path.  The passes below compute the weights on that set; a
// set that fails the rank test is routed to the global-memory path, which
// grows it as k_ls does.
constexpr int L3_CAP = 256;  // register rows (4 rows x 64 lanes) = the 3D staging segment

__global__ void __launch_bounds__(256) k_ls3_search(Geom g, Box b, const uint8_t* labels, CPDev cp, LSParams P,
                                                    int32_t* m_out, int32_t* grow_out, int32_t* st_idx,
                                                    uint8_t* route, int* err) {
    __shared__ int32_t list_idx[4][L3_CAP];
    __shared__ double list_r2[4][L3_CAP];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t ncs = cp.ncp * P.nsides;
    const int K = P.order_k;
    const int p = K * (K + 1) * (K + 2) / 6;
    const int64_t seg = L3_CAP;
    for (int64_t cs = (int64_t)blockIdx.x * 4 + wv; cs < ncs; cs += (int64_t)gridDim.x * 4) {
        const int64_t c = cs / P.nsides;
        const int sidx = (int)(cs % P.nsides);
        const uint8_t side = sidx == 0 ? K_PLUS : K_MINUS;
        double xc[3], nu[3];
        for (int d = 0; d < 3; ++d) {
            xc[d] = cp.x[d * cp.ncp + c];
            const double nd = cp.n[d * cp.ncp + c];
            nu[d] = sidx == 0 ? nd : -nd;
        }
        int result = 0;  // 0: none, 1: found, 2: routed
        for (int grow = 0; grow <= P.max_grow && result == 0; ++grow) {
            const double a = P.a0 + 0.5 * grow, bb = P.b0 + 0.5 * grow;
            const int R = (int)ceil(fmax(a, bb)) + 1;
            int wlo[3], wlen[3];
            for (int d = 0; d < 3; ++d) {
                int ci = (int)floor((xc[d] - g.lo) / g.h + 0.5);
                int lo = g.periodic ? ci - R : max(0, ci - R), hi = g.periodic ? ci + R : min(g.n, ci + R);
                wlo[d] = lo;
                wlen[d] = hi - lo + 1;
            }
            const int total = wlen[0] * wlen[1] * wlen[2];
            int count = 0;
            for (int base = 0; base < total; base += 64) {
                const int t = base + lane;
                bool keep = false;
                int32_t lidx = 0;
                double r2 = 0.0;
                if (t < total) {
                    const int q01 = t / wlen[0];
                    int ijk[3] = {wlo[0] + (t - q01 * wlen[0]), wlo[1] + q01 % wlen[1], wlo[2] + q01 / wlen[1]};
                    int wk3[3] = {ijk[0], ijk[1], ijk[2]};
                    if (g.periodic)
                        for (int d = 0; d < 3; ++d) wk3[d] = wrap_index(ijk[d], g.n);
                    bool inbox = true;
                    for (int d = 0; d < 3; ++d) inbox = inbox && wk3[d] >= b.lo[d] && wk3[d] < b.lo[d] + b.dims[d];
                    if (inbox) {
                        lidx = (int32_t)b.idx(wk3[0], wk3[1], wk3[2]);
                        if ((labels[lidx] & KIND_MASK) == side) {
#pragma clang fp contract(off)
                            double nn = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                double delta = (node_coord(g, ijk[d]) - xc[d]) / g.h;
                                nn += delta * nu[d];
                                r2 += delta * delta;
                            }
                            double tt = fmax(r2 - nn * nn, 0.0);
                            keep = (nn >= -SET_TOL) && (tt / (a * a) + nn * nn / (bb * bb) <= 1.0 + SET_TOL);
                        }
                    }
                }
                unsigned long long mask = __ballot(keep);
                int before = __popcll(mask & ((1ull << lane) - 1ull));
                if (keep && count + before < L3_CAP) {
                    list_idx[wv][count + before] = lidx;
                    list_r2[wv][count + before] = r2;
                }
                count += __popcll(mask);
            }
            if (count > L3_CAP) {  // too large for the register kernel
                result = 2;
                break;
            }
            if (count < p) continue;  // too few points (or none): grow
            // closest candidate: minimal r2, ties within SET_TOL to the lowest position
            double dmin = 1e300;
            for (int i = lane; i < count; i += 64) dmin = fmin(dmin, list_r2[wv][i]);
            dmin = wave_min(dmin);
            int closest = count;
            for (int i = lane; i < count; i += 64)
                if (list_r2[wv][i] <= dmin + SET_TOL) closest = min(closest, i);
            for (int off = 32; off > 0; off >>= 1) closest = min(closest, __shfl_xor(closest, off, 64));
            for (int i = lane; i < count - 1; i += 64) st_idx[cs * seg + i] = list_idx[wv][i + (i >= closest ? 1 : 0)];
            if (lane == 0) {
                m_out[cs] = count - 1;
                grow_out[cs] = grow;
            }
            result = 1;
        }
        if (lane == 0) {
            if (result == 2) {
                route[cs] = 1;
                grow_out[cs] = -3;
                m_out[cs] = 0;
            } else if (result == 0) {
                m_out[cs] = 0;
                grow_out[cs] = -1;
                atomicOr(err, 128);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The same fits by the corrected semi-normal equations, in five passes.  The
// weights are s = A (A^T A)^{-1} E^T, the minimum-norm solution of A^T s = E^T
// and the same s as Q R^{-T} E^T from A = QR.  A^T A is assembled from the 165
// moments sum_r x^a y^b z^c (a + b + c <= 8) of the set and factored by
// Cholesky (L_ii = |R_ii|, so the rank test reads the same diagonal as k_ls's
// QR); the semi-normal solution s0 = A G^{-1} E^T is corrected once with the
// residual E^T - A^T s0, which brings its error to the order of a Householder
// solution's (about eps cond(A)).  Passes over rows (lanes own rows, four
// each) alternate with passes over monomials (lane i owns row i of G);
// the per-fit intermediates live in global memory:
//   1. k_ls3_moments     rows       -> moments
//   2. k_ls3_chol        monomials  -> L (over the moments), e (the rank test;
//                                      near-singular fits go to the Householder
//                                      path)
//   3. k_ls3_resolve     monomials  -> z = G^{-1} e
//   4. k_ls3_rows        rows       -> s0 = A z, rho = e - A^T s0
//   5. k_ls3_resolve     monomials  -> z + dz, dz = G^{-1} rho
//   6. k_ls3_rows        rows       -> s = A (z + dz) = s0 + A dz
constexpr int MOM_N = 165;
constexpr int CS_NZ = 4 * 35;   // coefficient / residual entries per fit
constexpr int L_PACK = 35 * 36 / 2;  // packed lower triangle of L (the moments' slot)
// packed L: column t holds L_it for i = t..34 (1 / L_tt in place of L_tt)
__host__ __device__ constexpr int lpack_col(int t) { return 35 * t - t * (t - 1) / 2; }

// exponents of the 35 monomials of total degree <= 4 in 3D, in the order of
// monomials(): degree t, then i = t..0, then j = t-i..0, k = t-i-j
struct Mono3 {
    int e[35][3];
};
constexpr Mono3 mono3_table() {
    Mono3 m{};
    int c = 0;
    for (int t = 0; t <= 4; ++t)
        for (int i = t; i >= 0; --i)
            for (int j = t - i; j >= 0; --j) {
                m.e[c][0] = i;
                m.e[c][1] = j;
                m.e[c][2] = t - i - j;
                ++c;
            }
    return m;
}
constexpr Mono3 MONO3 = mono3_table();
// moments grouped by the z power c; inside a group by s = a + b, then by b
constexpr int MOM_OFF[10] = {0, 45, 81, 109, 130, 145, 155, 161, 164, 165};
__device__ inline int mom_index(int a, int b, int c) {
    const int s = a + b;
    int off = 0;
    for (int cc = 0; cc < c; ++cc) off += (9 - cc) * (10 - cc) / 2;
    return off + s * (s + 1) / 2 + b;
}

// the lane's rows of a fit: offsets (x - x_c) / sc and a 0/1 weight (row 0 = x_c)
template <int NR>
__device__ inline void ls3_rows(const Geom& g, const Box& b, const int32_t* st, int M, const double* xc, double sc,
                                int lane, double (*X)[3], double* wt) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int r = lane + 64 * q;
        X[q][0] = X[q][1] = X[q][2] = 0.0;
        wt[q] = r < M ? 1.0 : 0.0;
        if (r > 0 && r < M) {
            int ijk[3];
            b.coords(st[r - 1], ijk);
            for (int d = 0; d < 3; ++d) X[q][d] = (node_coord(g, unwrap_near(g, ijk[d], xc[d])) - xc[d]) / sc;
        }
    }
}

template <int CTRL>
__device__ inline double quad_copy(double v) {  // every lane of a quad is a source: no old value needed
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffffll), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// wave sums of v[0..NV) written to out[0..NV) (global or LDS): quads add by
// DPP, the 16 quad sums of each value go to LDS, lane j adds those of value j
// in a fixed order.  One wavefront per block: __syncthreads orders the LDS use.
template <int NV>
__device__ inline void ls3_wave_sums(double (*part)[16], int lane, const double* v, double* out) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double x = v[j];
        x += quad_copy<0xB1>(x);  // quad_perm [1, 0, 3, 2]
        x += quad_copy<0x4E>(x);  // quad_perm [2, 3, 0, 1]
        if ((lane & 3) == 0) part[j][lane >> 2] = x;
    }
    __syncthreads();
    if (lane < NV) {
        const double* p = part[lane];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int i = 0; i < 16; i += 4) {
            a0 += p[i];
            a1 += p[i + 1];
            a2 += p[i + 2];
            a3 += p[i + 3];
        }
        out[lane] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
}

// the moments of one z power CZ: x^a y^b z^CZ, a + b <= 8 - CZ (pz holds z^CZ
// times the row weight on entry, z^(CZ+1) times it on return)
template <int NR, int CZ>
__device__ inline void ls3_moment_group(double (*part)[16], int lane, const double (*X)[3], double* pz,
                                        double* mom) {
    constexpr int m = 8 - CZ, NV = (m + 1) * (m + 2) / 2;
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        double px[m + 1], py[m + 1];
        px[0] = py[0] = 1.0;
#pragma unroll
        for (int e = 1; e <= m; ++e) {
            px[e] = px[e - 1] * X[q][0];
            py[e] = py[e - 1] * X[q][1];
        }
#pragma unroll
        for (int a = 0; a <= m; ++a) {
            const double pxz = px[a] * pz[q];
#pragma unroll
            for (int bb = 0; a + bb <= m; ++bb) {
                const int sidx = a + bb;
                acc[sidx * (sidx + 1) / 2 + bb] += pxz * py[bb];
            }
        }
        pz[q] *= X[q][2];
        __builtin_amdgcn_sched_barrier(0);  // one row's powers live at a time
    }
    ls3_wave_sums<NV>(part, lane, acc, mom + MOM_OFF[CZ]);
}

// pass 1: the 165 moments of every fit's set, one z power at a time
template <int NR>
__global__ void __launch_bounds__(64) k_ls3_moments(Geom g, Box b, CPDev cp, LSParams P, const int32_t* m_out,
                                                    const int32_t* grow_out, const int32_t* st_idx, double* mom) {
    __shared__ double part[45][16];
    const int lane = threadIdx.x;
    const int64_t ncs = cp.ncp * P.nsides;
    for (int64_t cs = blockIdx.x; cs < ncs; cs += gridDim.x) {
        const int grow = grow_out[cs];
        if (grow < 0) continue;  // routed or failed in the search
        const int64_t c = cs / P.nsides;
        double xc[3];
        for (int d = 0; d < 3; ++d) xc[d] = cp.x[d * cp.ncp + c];
        double X[NR][3], wt[NR];
        ls3_rows<NR>(g, b, st_idx + cs * L3_CAP, m_out[cs] + 1, xc, (P.a0 + 0.5 * grow) * g.h, lane, X, wt);
        double pz[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) pz[q] = wt[q];
        ls3_moment_group<NR, 0>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 1>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 2>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 3>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 4>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 5>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 6>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 7>(part, lane, X, pz, mom + cs * L_PACK);
        ls3_moment_group<NR, 8>(part, lane, X, pz, mom + cs * L_PACK);
    }
}

// G z = e for up to four right-hand sides (e: lane i holds entry i) with G =
// L L^T, from the scaled triangles in one array: T[t][i] = L_it / L_ii below
// the diagonal (i > t) and L_ti / L_ii above it (i < t); di = 1 / L_ii in lane
// i; z0 + z to zc[k][i].  Lane i carries its entry divided by L_ii, so that it is
// final (y_i, then z_i) once step i is reached and every step is one broadcast
// and one FMA per right-hand side; lanes past 34 carry values nobody reads.
__device__ __forceinline__ void ls3_solves(int lane, int nrows, const double (*T)[35], double di, const double* e,
                                           const double* z0, double* zc) {
    const int lm = lane < 35 ? lane : 34;
    double c0 = e[0] * di, c1 = e[1] * di, c2 = e[2] * di, c3 = e[3] * di;
#pragma unroll 7
    for (int t = 0; t < 35; ++t) {  // L y = e
        const double f = lane > t ? T[t][lm] : 0.0;
        const double y0 = lane_value(c0, t), y1 = lane_value(c1, t), y2 = lane_value(c2, t),
                     y3 = lane_value(c3, t);
        c0 = fma(-f, y0, c0);
        c1 = fma(-f, y1, c1);
        c2 = fma(-f, y2, c2);
        c3 = fma(-f, y3, c3);
    }
    c0 *= di;
    c1 *= di;
    c2 *= di;
    c3 *= di;
#pragma unroll 7
    for (int t = 34; t >= 0; --t) {  // L^T z = y
        const double bt = lane < t ? T[t][lm] : 0.0;
        const double z0 = lane_value(c0, t), z1 = lane_value(c1, t), z2 = lane_value(c2, t),
                     z3 = lane_value(c3, t);
        c0 = fma(-bt, z0, c0);
        c1 = fma(-bt, z1, c1);
        c2 = fma(-bt, z2, c2);
        c3 = fma(-bt, z3, c3);
    }
    if (lane < 35) {
        double* z = zc + lane;
        if (nrows > 0) z[0] = z0[0] + c0;
        if (nrows > 1) z[35] = z0[1] + c1;
        if (nrows > 2) z[70] = z0[2] + c2;
        if (nrows > 3) z[105] = z0[3] + c3;
    }
}

// pass 2: G = L L^T by Cholesky (lane i holds row i of G; column k of L
// broadcast through LDS) and the rank test; the packed L goes over the fit's
// moments and the functionals e (ghost values, d/dn, d/dx_d at x_c) to rho
__global__ void __launch_bounds__(64) k_ls3_chol(Geom g, Box b, CPDev cp, LSParams P, int32_t* m_out,
                                                 int32_t* grow_out, uint8_t* route, double* mom, double* rho) {
    __shared__ double col[64];
    __shared__ double cube[9 * 9 * 9];  // moment (a, b, c) at a + 9 b + 81 c
    const int lane = threadIdx.x;
    const int64_t ncs = cp.ncp * P.nsides;
    const int nrows = P.nrows;
    const int li = lane < 35 ? lane : 0;
    // G_ij is the moment of exponents e_i + e_j: lane i reads row i at fixed
    // offsets from its own base
    const int ea = lane < 35 ? MONO3.e[li][0] : 0, eb = lane < 35 ? MONO3.e[li][1] : 0,
              ec = lane < 35 ? MONO3.e[li][2] : 0;
    const int gbase = ea + 9 * eb + 81 * ec;
    int cpos[3];  // cube positions of the moments this lane moves
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int m = lane + 64 * q;
        int c = 0;
        while (c < 8 && m >= MOM_OFF[c + 1]) ++c;
        const int r = m - MOM_OFF[c];
        int sab = 0;
        while ((sab + 1) * (sab + 2) / 2 <= r) ++sab;
        const int bb = r - sab * (sab + 1) / 2;
        cpos[q] = m < MOM_N ? (sab - bb) + 9 * bb + 81 * c : -1;
    }
    for (int64_t cs = blockIdx.x; cs < ncs; cs += gridDim.x) {
        const int grow = grow_out[cs];
        if (grow < 0) continue;
        double* mm = mom + cs * L_PACK;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (cpos[q] >= 0) cube[cpos[q]] = mm[lane + 64 * q];
        __syncthreads();
        double Lr[35];
#pragma unroll
        for (int j = 0; j < 35; ++j)
            Lr[j] = lane < 35 ? cube[gbase + MONO3.e[j][0] + 9 * MONO3.e[j][1] + 81 * MONO3.e[j][2]] : 0.0;
        double rmax = 0.0, rmin = 1e300, di = 0.0;  // di = 1 / L_ii in lane i
        bool pd = true;
#pragma unroll
        for (int k = 0; k < 35; ++k) {
            const double dkk = lane_value(Lr[k], k);
            pd = pd && dkk > 0.0;
            // 1 / sqrt by the hardware estimate and two Newton steps
            // (y <- y + y (1 - d y^2) / 2), then L_kk = d / sqrt(d)
            const double dd = fmax(dkk, 1e-300);
            double inv = __builtin_amdgcn_rsq(dd);
#pragma unroll
            for (int it = 0; it < 2; ++it) inv = fma(0.5 * inv, fma(-dd * inv, inv, 1.0), inv);
            const double lkk = dd * inv;
            rmax = fmax(rmax, lkk);
            rmin = fmin(rmin, lkk);
            if (lane == k) di = inv;
            Lr[k] = lane == k ? lkk : Lr[k] * inv;
            if (k == 34) break;
            col[lane] = Lr[k];
            __syncthreads();
            // all lanes update: entries above the diagonal (lane < j) take
            // values that are never read
#pragma unroll
            for (int j = k + 1; j < 35; ++j) Lr[j] -= Lr[k] * col[j];
            __syncthreads();
        }
        if (!pd || rmin < 1e-6 * rmax) {  // near rank deficient: the Householder path decides
            if (lane == 0) {
                route[cs] = 1;
                grow_out[cs] = -3;
                m_out[cs] = 0;
            }
            __syncthreads();
            continue;
        }
        if (lane < 35) {
#pragma unroll
            for (int t = 0; t < 35; ++t)  // packed L (1 / L_tt on the diagonal) over the moments, all read by now
                if (t <= lane) mm[lpack_col(t) + lane - t] = t < lane ? Lr[t] : di;
        }
        double* rk = rho + cs * CS_NZ;
        {
            if (lane < 35) {  // the functionals, entry = monomial
                const int64_t c = cs / P.nsides;
                const int sidx = (int)(cs % P.nsides);
                const double sc = (P.a0 + 0.5 * grow) * g.h;
                double xc[3];
                for (int d = 0; d < 3; ++d) xc[d] = cp.x[d * cp.ncp + c];
                const int axis = cp.axis[c];
                const int64_t anode = cp.a[sidx * cp.ncp + c];
                const int adir = cp.dir[sidx * cp.ncp + c];
                int acoord[3];
                b.coords(anode, acoord);
                double xa[3];
                for (int d = 0; d < 3; ++d) xa[d] = node_coord(g, unwrap_near(g, acoord[d], xc[d]));
                for (int k = 0; k < nrows && k < 4; ++k) {
                    double val;
                    if (k < P.w) {
                        double xg[3] = {xa[0], xa[1], xa[2]};
                        xg[axis] = xa[axis] + (double)((k + 1) * adir) * g.h;
                        double xi[3];
                        for (int d = 0; d < 3; ++d) xi[d] = (xg[d] - xc[d]) / sc;
                        val = ipow(xi[0], ea) * ipow(xi[1], eb) * ipow(xi[2], ec);
                    } else {
                        // row w: d/dn; rows w + 1 + d: d/dx_d (gradient fits)
                        val = 0.0;
                        if (ea + eb + ec == 1) {
                            const int d = ea ? 0 : (eb ? 1 : 2);
                            const int r = k - P.w;
                            val = (r == 0 ? cp.n[d * cp.ncp + c] : (d == r - 1 ? 1.0 : 0.0)) / sc;
                        }
                    }
                    rk[k * 35 + lane] = val;
                }
            }
        }
        __syncthreads();
    }
}

// G z = rhs from the L that the Cholesky pass stored: z = G^{-1} e (rhs = e,
// before the rows pass) and z + dz with dz = G^{-1} rho (after it, add = 1)
__global__ void __launch_bounds__(64) k_ls3_resolve(CPDev cp, LSParams P, const int32_t* grow_out,
                                                    const double* mom, const double* rho, double* zc, int add) {
    __shared__ double Ts[35][35];
    const int lane = threadIdx.x;
    const int li = lane < 35 ? lane : 0;
    const int64_t ncs = cp.ncp * P.nsides;
    const int nrows = P.nrows;
    for (int64_t cs = blockIdx.x; cs < ncs; cs += gridDim.x) {
        if (grow_out[cs] < 0) continue;
        const double* mm = mom + cs * L_PACK;
        double di = 0.0;
        if (lane < 35) {
            // lane i: L_it from column t (t < i), L_ti from column i (t >= i;
            // t = i reads 1 / L_ii); all loads in flight before the first use
            double v[35];
#pragma unroll
            for (int t = 0; t < 35; ++t) v[t] = mm[t < li ? lpack_col(t) + li - t : lpack_col(li) + t - li];
            di = mm[lpack_col(li)];
#pragma unroll
            for (int t = 0; t < 35; ++t) Ts[t][lane] = t == lane ? 0.0 : v[t] * di;
        }
        double e[4] = {0.0, 0.0, 0.0, 0.0}, z0[4] = {0.0, 0.0, 0.0, 0.0};
        const double* rk = rho + cs * CS_NZ;
        if (lane < 35)
            for (int k = 0; k < nrows && k < 4; ++k) {
                e[k] = rk[k * 35 + lane];
                if (add) z0[k] = zc[cs * CS_NZ + k * 35 + lane];
            }
        __syncthreads();
        ls3_solves(lane, nrows, Ts, di, e, z0, zc + cs * CS_NZ);
        __syncthreads();
    }
}

// passes 4 and 6 over the rows of a fit: pass 4 forms s0 = A z and from it rho
// = e - A^T s0 (in place of e); pass 6 writes s = A (z + dz), equal to s0 + A dz,
// into the staging weights (row 0 into Sc).  Every load of a fit is issued
// before its first use: with one wave per SIMD nothing else hides the latency.
template <int NR, bool second>
__global__ void __launch_bounds__(64) k_ls3_rows(Geom g, Box b, CPDev cp, LSParams P, const int32_t* m_out,
                                                 const int32_t* grow_out, const int32_t* st_idx, const double* zc,
                                                 double* rho, double* S_out, double* Sc_out) {
    __shared__ double part[35][16];
    __shared__ double zs[4][35];
    __shared__ double es[4][35];
    __shared__ double red[35];
    const int lane = threadIdx.x;
    const int li = lane < 35 ? lane : 0;
    const int64_t ncs = cp.ncp * P.nsides;
    const int nrows = P.nrows < 4 ? P.nrows : 4;
    const int64_t seg = L3_CAP, snz = ncs * seg;
    for (int64_t cs = blockIdx.x; cs < ncs; cs += gridDim.x) {
        const int grow = grow_out[cs];
        const int M = m_out[cs] + 1;
        const int64_t c = cs / P.nsides;
        double xc[3];
        for (int d = 0; d < 3; ++d) xc[d] = cp.x[d * cp.ncp + c];
        const int32_t* st = st_idx + cs * L3_CAP;
        int32_t node[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) node[q] = lane + 64 * q >= 1 ? st[lane + 64 * q - 1] : 0;
        double zk[4], ek[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            zk[k] = k < nrows ? zc[cs * CS_NZ + k * 35 + li] : 0.0;
            ek[k] = !second && k < nrows ? rho[cs * CS_NZ + k * 35 + li] : 0.0;
        }
        if (grow < 0) continue;
        if (lane < 35)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                zs[k][lane] = zk[k];
                es[k][lane] = ek[k];
            }
        const double sc = (P.a0 + 0.5 * grow) * g.h;
        double X[NR][3], wt[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) {  // the lane's rows: offsets (x - x_c) / sc, weight 1 (row 0 = x_c)
            const int r = lane + 64 * q;
            X[q][0] = X[q][1] = X[q][2] = 0.0;
            wt[q] = r < M ? 1.0 : 0.0;
            if (r > 0 && r < M) {
                int ijk[3];
                b.coords(node[q], ijk);
                for (int d = 0; d < 3; ++d) X[q][d] = (node_coord(g, unwrap_near(g, ijk[d], xc[d])) - xc[d]) / sc;
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < nrows; ++k) {
            if constexpr (!second) {
                // s0 = A z row by row and rho = e - A^T s0, each row's monomials
                // formed once for both
                double acc[35];
#pragma unroll
                for (int i = 0; i < 35; ++i) acc[i] = 0.0;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    double px[5], py[5], pz[5];
                    px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
                    for (int e = 1; e < 5; ++e) {
                        px[e] = px[e - 1] * X[q][0];
                        py[e] = py[e - 1] * X[q][1];
                        pz[e] = pz[e - 1] * X[q][2];
                    }
                    double mono[35];
#pragma unroll
                    for (int cc = 0; cc < 35; ++cc) mono[cc] = px[MONO3.e[cc][0]] * py[MONO3.e[cc][1]] * pz[MONO3.e[cc][2]];
                    double sv = 0.0;
#pragma unroll
                    for (int cc = 0; cc < 35; ++cc) sv += mono[cc] * zs[k][cc];
                    const double sq = sv * wt[q];
#pragma unroll
                    for (int i = 0; i < 35; ++i) acc[i] += mono[i] * sq;
                    __builtin_amdgcn_sched_barrier(0);
                }
                ls3_wave_sums<35>(part, lane, acc, red);
                if (lane < 35) rho[cs * CS_NZ + k * 35 + lane] = es[k][lane] - red[lane];
                continue;
            }
            double sv[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                double px[5], py[5], pz[5];
                px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
                for (int e = 1; e < 5; ++e) {
                    px[e] = px[e - 1] * X[q][0];
                    py[e] = py[e - 1] * X[q][1];
                    pz[e] = pz[e - 1] * X[q][2];
                }
                double acc = 0.0;
#pragma unroll
                for (int cc = 0; cc < 35; ++cc)
                    acc += px[MONO3.e[cc][0]] * py[MONO3.e[cc][1]] * pz[MONO3.e[cc][2]] * zs[k][cc];
                sv[q] = acc;
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (second) {
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const int r = lane + 64 * q;
                    if (r >= 1 && r < M)
                        S_out[(int64_t)k * snz + cs * seg + r - 1] = sv[q];
                    else if (r == 0)
                        Sc_out[cs * nrows + k] = sv[q];
                }
            } else {
                double acc[35];
#pragma unroll
                for (int i = 0; i < 35; ++i) acc[i] = 0.0;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    double px[5], py[5], pz[5];
                    px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
                    for (int e = 1; e < 5; ++e) {
                        px[e] = px[e - 1] * X[q][0];
                        py[e] = py[e - 1] * X[q][1];
                        pz[e] = pz[e - 1] * X[q][2];
                    }
                    const double sq = sv[q] * wt[q];
#pragma unroll
                    for (int i = 0; i < 35; ++i)
                        acc[i] += px[MONO3.e[i][0]] * py[MONO3.e[i][1]] * pz[MONO3.e[i][2]] * sq;
                    __builtin_amdgcn_sched_barrier(0);
                }
                ls3_wave_sums<35>(part, lane, acc, red);
                if (lane < 35) rho[cs * CS_NZ + k * 35 + lane] = es[k][lane] - red[lane];
            }
        }
        __syncthreads();
    }
}

void run_ls3_csne(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp, const LSParams& P,
                  int32_t* m_out, int32_t* grow_out, int32_t* st_idx, double* S, double* Sc, uint8_t* route,
                  double* mom, double* zc, double* rho, int* d_err, hipStream_t s) {
    const int64_t ncs = cp.ncp * P.nsides;
    if (ncs == 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>(ncs, 65536);
    hipLaunchKernelGGL(k_ls3_search, dim3(cdiv(ncs, 4)), dim3(256), 0, s, g, b, labels, cp, P, m_out, grow_out,
                       st_idx, route, d_err);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_ls3_moments<L3_CAP / 64>), dim3(blocks), dim3(64), 0, s, g, b, cp, P, m_out, grow_out,
                       st_idx, mom);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ls3_chol, dim3(blocks), dim3(64), 0, s, g, b, cp, P, m_out, grow_out, route, mom, rho);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ls3_resolve, dim3(blocks), dim3(64), 0, s, cp, P, grow_out, mom, rho, zc, 0);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_ls3_rows<L3_CAP / 64, false>), dim3(blocks), dim3(64), 0, s, g, b, cp, P, m_out, grow_out, st_idx,
                       zc, rho, S, Sc);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ls3_resolve, dim3(blocks), dim3(64), 0, s, cp, P, grow_out, mom, rho, zc, 1);
    IIM_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_ls3_rows<L3_CAP / 64, true>), dim3(blocks), dim3(64), 0, s, g, b, cp, P, m_out, grow_out, st_idx,
                       zc, rho, S, Sc);
    IIM_LAUNCH_CHECK();
}
int64_t ls3_csne_doubles_per_fit() { return L_PACK + 2 * CS_NZ; }

// staging (fixed segments of seg entries per fit) -> CSR, for the fits of the
// register path (route[cs] == 0); one wavefront per fit
__global__ void __launch_bounds__(256) k_ls_compact(int64_t ncs, int seg, int nrows, const int32_t* m,
                                                    const uint8_t* route, const int64_t* ptr, const int32_t* st_idx,
                                                    const double* st_S, int32_t* idx, double* S) {
    const int lane = threadIdx.x & 63;
    const int64_t nnz = ptr[ncs], snz = ncs * (int64_t)seg;
    for (int64_t cs = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / 64; cs < ncs;
         cs += (int64_t)gridDim.x * blockDim.x / 64) {
        if (route[cs]) continue;
        const int64_t src = cs * seg, dst = ptr[cs];
        for (int r = lane; r < m[cs]; r += 64) {
            idx[dst + r] = st_idx[src + r];
            for (int k = 0; k < nrows; ++k) S[(int64_t)k * nnz + dst + r] = st_S[(int64_t)k * snz + src + r];
        }
    }
}

void run_ls_compact(int64_t ncs, int seg, int nrows, const int32_t* m, const uint8_t* route, const int64_t* ptr,
                    const int32_t* st_idx, const double* st_S, int32_t* idx, double* S, hipStream_t s) {
    if (ncs == 0) return;
    const int blocks = (int)std::min<int64_t>(cdiv(ncs * 64, 256), 8192);
    hipLaunchKernelGGL(k_ls_compact, dim3(blocks), dim3(256), 0, s, ncs, seg, nrows, m, route, ptr, st_idx, st_S, idx,
                       S);
    IIM_LAUNCH_CHECK();
}

int ls_segment(int dim) { return dim == 2 ? 64 * 2 : 64 * 4; }

void run_ls(const Geom& g, const Box& b, const uint8_t* labels, const CPDev& cp, const LSParams& P, int pass,
            int32_t* m_out, int32_t* grow_out, const int64_t* ptr, int32_t* idx, double* S, double* Sc,
            double* scratch, int64_t scratch_waves, int* d_err, const int32_t* cs_list, int64_t n_list,
            uint8_t* route, hipStream_t s) {
    int64_t ncs = cp.ncp * P.nsides;
    int64_t nwork = cs_list ? n_list : ncs;
    if (nwork == 0) return;
    int blocks = (int)std::min<int64_t>(nwork, cs_list ? scratch_waves : 4096);
    if (g.dim == 2 && P.order_k == 7)
        hipLaunchKernelGGL((k_ls<28, 2>), dim3(blocks), dim3(64), 0, s, g, b, labels, cp, P, pass, m_out, grow_out, ptr,
                           idx, S, Sc, scratch, d_err, cs_list, n_list, route);
    else if (g.dim == 2)
        hipLaunchKernelGGL((k_ls<15, 2>), dim3(blocks), dim3(64), 0, s, g, b, labels, cp, P, pass, m_out, grow_out, ptr,
                           idx, S, Sc, scratch, d_err, cs_list, n_list, route);
    else
        hipLaunchKernelGGL((k_ls<35, 4>), dim3(blocks), dim3(64), 0, s, g, b, labels, cp, P, pass, m_out, grow_out, ptr,
                           idx, S, Sc, scratch, d_err, cs_list, n_list, route);
    IIM_LAUNCH_CHECK();
}

}  // namespace iim
