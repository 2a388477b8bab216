// Internal definitions shared by the HIP kernels and the host core.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "iim.h"

namespace iim {

// ---------------------------------------------------------------------------
// errors: host code throws Error; the C ABI converts it to a status code
// ---------------------------------------------------------------------------
struct Error : public std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define IIM_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::iim::Error(IIM_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

#define IIM_LAUNCH_CHECK() IIM_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// node labels: kind in bits 0-1, flags above
// ---------------------------------------------------------------------------
enum : uint8_t { K_INACTIVE = 0, K_PLUS = 1, K_MINUS = 2, K_BOX = 3 };
constexpr uint8_t KIND_MASK = 3;
constexpr uint8_t F_HO_IRR = 4;  // high-order stencil needs ghost or box values
constexpr uint8_t F_SW_IRR = 8;  // Shortley-Weller row differs from the 5/7-point one

__host__ __device__ inline bool is_unknown(uint8_t lab) {
    uint8_t k = lab & KIND_MASK;
    return k == K_PLUS || k == K_MINUS;
}

// ---------------------------------------------------------------------------
// storage box of a level: a padded bounding box of its unknowns, x fastest
// ---------------------------------------------------------------------------
struct Box {
    int lo[3];
    int dims[3];
    __host__ __device__ int64_t size() const { return (int64_t)dims[0] * dims[1] * dims[2]; }
    __host__ __device__ int64_t idx(int i, int j, int k) const {
        return (int64_t)(i - lo[0]) + (int64_t)dims[0] * ((int64_t)(j - lo[1]) + (int64_t)dims[1] * (k - lo[2]));
    }
    __host__ __device__ int64_t stride(int d) const {
        return d == 0 ? 1 : (d == 1 ? (int64_t)dims[0] : (int64_t)dims[0] * dims[1]);
    }
    __host__ __device__ void coords(int64_t l, int* ijk) const {
        if (l >= 0 && l <= 0x7fffffff) {  // 32-bit division: a fraction of the 64-bit sequence
            const uint32_t u = (uint32_t)l, d0 = (uint32_t)dims[0], d1 = (uint32_t)dims[1];
            const uint32_t r = u / d0;
            ijk[0] = (int)(u - r * d0) + lo[0];
            ijk[1] = (int)(r % d1) + lo[1];
            ijk[2] = (int)(r / d1) + lo[2];
            return;
        }
        ijk[0] = (int)(l % dims[0]) + lo[0];
        int64_t r = l / dims[0];
        ijk[1] = (int)(r % dims[1]) + lo[1];
        ijk[2] = (int)(r / dims[1]) + lo[2];
    }
};

// ---------------------------------------------------------------------------
// geometry on one grid level
// ---------------------------------------------------------------------------
struct Geom {
    int kind;       // IIM_GEOM_*
    int side;       // IIM_SIDE_*
    int dim;
    int n;          // intervals of this level
    double lo, h;   // node i at lo + i * h
    const double* p;  // device copy of the parameters
    int periodic;   // 1: periodic in every direction (node n is node 0's image, not stored)
};

// index i taken into 0..n-1
__host__ __device__ inline int wrap_index(int i, int n) {
    const int r = i % n;
    return r < 0 ? r + n : r;
}
// the same for -n <= i < 2n (neighbour offsets below the period): no division
__host__ __device__ inline int wrap_near(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ inline double node_coord(const Geom& g, int i) {
#pragma clang fp contract(off)
    return g.lo + (double)i * g.h;
}

// sign of phi for one sphere [c..., r]: squared distance summed x, y, z first
__device__ inline int sphere_sign(const double* c, double r, int dim, const double* x) {
#pragma clang fp contract(off)
    double d2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        double t = x[d] - c[d];
        d2 = d2 + t * t;
    }
    double q = d2 - r * r;
    return q < 0.0 ? -1 : (q > 0.0 ? 1 : 0);
}

// Chebyshev T_L(c) and U_{L-1}(c) by three-term recurrences
__device__ inline void cheb_tu(int L, double c, double* T, double* U) {
#pragma clang fp contract(off)
    double t0 = 1.0, t1 = c;
    for (int i = 0; i < L - 1; ++i) {
        double t2 = 2.0 * c * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    *T = (L == 0) ? 1.0 : t1;
    double u0 = 1.0, u1 = 2.0 * c;
    for (int i = 0; i < L - 2; ++i) {
        double u2 = 2.0 * c * u1 - u0;
        u0 = u1;
        u1 = u2;
    }
    *U = (L <= 1) ? (L == 1 ? 1.0 : 0.0) : u1;
}

// phi = rho - (r0 + eps T_L(dx/rho)) for the star
__device__ inline double star_phi(const double* p, double x, double y) {
#pragma clang fp contract(off)
    double dx = x - p[0];
    double dy = y - p[1];
    double rho = sqrt(dx * dx + dy * dy);
    double c = rho > 0.0 ? dx / rho : 1.0;
    int L = (int)llround(p[4]);
    double t0 = 1.0, t1 = c;
    for (int i = 0; i < L - 1; ++i) {
        double t2 = 2.0 * c * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    double t = L >= 1 ? t1 : 1.0;
    return rho - (p[2] + p[3] * t);
}

__device__ inline int sgn(double v) { return v < 0.0 ? -1 : (v > 0.0 ? 1 : 0); }

// sin t and cos t from IEEE basic operations only, so that every
// implementation of these steps rounds them identically: Cody-Waite reduction
// r = t - q pi/2 (pi/2 split into three parts, q the nearest integer of
// t 2/pi), then the Taylor series of sin and cos on |r| <= pi/4 to degree 19
// and 18 in Horner form, and the quadrant q mod 4.  Accurate to about 2 ulp.
__device__ inline void det_sincos(double t, double* sn, double* cs) {
#pragma clang fp contract(off)
    const double q = floor(t * 0.6366197723675814 + 0.5);
    const double r = ((t - q * 1.570796325802803) - q * 9.920935791635221e-10) - q * 5.170182981794105e-19;
    const double z = r * r;
    double ps = -8.22063524662433e-18;
    ps = 2.8114572543455206e-15 + z * ps;
    ps = -7.647163731819816e-13 + z * ps;
    ps = 1.6059043836821613e-10 + z * ps;
    ps = -2.505210838544172e-08 + z * ps;
    ps = 2.7557319223985893e-06 + z * ps;
    ps = -0.0001984126984126984 + z * ps;
    ps = 0.008333333333333333 + z * ps;
    ps = -0.16666666666666666 + z * ps;
    const double s0 = r + r * (z * ps);
    double pc = -1.5619206968586225e-16;
    pc = 4.779477332387385e-14 + z * pc;
    pc = -1.1470745597729725e-11 + z * pc;
    pc = 2.08767569878681e-09 + z * pc;
    pc = -2.755731922398589e-07 + z * pc;
    pc = 2.48015873015873e-05 + z * pc;
    pc = -0.001388888888888889 + z * pc;
    pc = 0.041666666666666664 + z * pc;
    pc = -0.5 + z * pc;
    const double c0 = 1.0 + z * pc;
    double m = fmod(q, 4.0);
    if (m < 0.0) m += 4.0;
    if (m == 0.0) {
        *sn = s0;
        *cs = c0;
    } else if (m == 1.0) {
        *sn = c0;
        *cs = -s0;
    } else if (m == 2.0) {
        *sn = -s0;
        *cs = -c0;
    } else {
        *sn = -c0;
        *cs = s0;
    }
}

// gyroid: phi = cos(k1 x) sin(k2 y) + cos(k2 y) sin(k3 z) + cos(k3 z) sin(k1 x) - alpha,
// p = [k1, k2, k3, alpha]; the solved region is phi > 0 (exterior side).  Summed
// left to right, sin and cos by det_sincos.
__device__ inline double gyroid_phi(const double* p, const double* x) {
#pragma clang fp contract(off)
    double sx, cx, sy, cy, sz, cz;
    det_sincos(p[0] * x[0], &sx, &cx);
    det_sincos(p[1] * x[1], &sy, &cy);
    det_sincos(p[2] * x[2], &sz, &cz);
    return ((cx * sy + cy * sz) + cz * sx) - p[3];
}

__device__ inline void gyroid_grad(const double* p, const double* x, double* g) {
    double sx, cx, sy, cy, sz, cz;
    det_sincos(p[0] * x[0], &sx, &cx);
    det_sincos(p[1] * x[1], &sy, &cy);
    det_sincos(p[2] * x[2], &sz, &cz);
    g[0] = -p[0] * sx * sy + p[0] * cz * cx;
    g[1] = p[1] * cx * cy - p[1] * sy * sz;
    g[2] = p[2] * cy * cz - p[2] * sz * sx;
}

// largest absolute principal curvature of the gyroid's level surface at x:
// the non-normal eigenvalues of P Hess P / |grad| (P the tangent projector),
// from the trace and the sum of the principal 2 x 2 minors
__device__ inline double gyroid_curvature(const double* p, const double* x) {
    double sx, cx, sy, cy, sz, cz;
    det_sincos(p[0] * x[0], &sx, &cx);
    det_sincos(p[1] * x[1], &sy, &cy);
    det_sincos(p[2] * x[2], &sz, &cz);
    double g[3];
    gyroid_grad(p, x, g);
    double H[3][3];
    H[0][0] = -p[0] * p[0] * cx * sy - p[0] * p[0] * cz * sx;
    H[1][1] = -p[1] * p[1] * cx * sy - p[1] * p[1] * cy * sz;
    H[2][2] = -p[2] * p[2] * cy * sz - p[2] * p[2] * cz * sx;
    H[0][1] = H[1][0] = -p[0] * p[1] * sx * cy;
    H[1][2] = H[2][1] = -p[1] * p[2] * sy * cz;
    H[0][2] = H[2][0] = -p[0] * p[2] * sz * cx;
    const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double nv[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
    double P[3][3], T[3][3], Sh[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[a][b] = (a == b ? 1.0 : 0.0) - nv[a] * nv[b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int c = 0; c < 3; ++c) t += P[a][c] * H[c][b];
            T[a][b] = t;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int c = 0; c < 3; ++c) t += T[a][c] * P[c][b];
            Sh[a][b] = t / gn;
        }
    const double tr = Sh[0][0] + Sh[1][1] + Sh[2][2];
    const double m2 = Sh[0][0] * Sh[1][1] - Sh[0][1] * Sh[1][0] + Sh[0][0] * Sh[2][2] - Sh[0][2] * Sh[2][0] +
                      Sh[1][1] * Sh[2][2] - Sh[1][2] * Sh[2][1];
    const double half = 0.5 * tr;
    return fabs(half) + sqrt(fmax(half * half - m2, 0.0));
}

// sign of phi (-1 inside the body, 0 on Gamma, +1 outside)
// sign of the level set at x for a DIM known at compile time; p: the
// parameters (g.p, or a copy of them staged by the caller)
template <int DIM>
__device__ inline int geom_sign_d(const Geom& g, const double* p, const double* x) {
    if (g.kind == IIM_GEOM_SPHERE) return sphere_sign(p, p[DIM], DIM, x);
    if (g.kind == IIM_GEOM_GYROID) return sgn(gyroid_phi(p, x));
    if (g.kind == IIM_GEOM_STAR2D) return sgn(star_phi(p, x[0], x[1]));
    int cnt = (int)llround(p[0]);
    bool on = false;
    for (int s = 0; s < cnt; ++s) {
        const double* q = p + 1 + (DIM + 1) * s;
        int v = sphere_sign(q, q[DIM], DIM, x);
        if (v < 0) return -1;
        if (v == 0) on = true;
    }
    return on ? 0 : 1;
}
__device__ inline int geom_sign(const Geom& g, const double* x) {
    return g.dim == 3 ? geom_sign_d<3>(g, g.p, x) : geom_sign_d<2>(g, g.p, x);
}

// kind of a node of the level (box faces included), or 255 = rejected
template <int DIM>
__device__ inline uint8_t node_kind_d(const Geom& g, const double* p, const int* ijk) {
    double x[3] = {0.0, 0.0, 0.0};
    bool face = false;
    if (g.periodic) {
        // no box faces; the image planes (index n) hold no unknowns
        for (int d = 0; d < DIM; ++d) {
            if (ijk[d] >= g.n) return K_INACTIVE;
            x[d] = node_coord(g, ijk[d]);
        }
        const int s = geom_sign_d<DIM>(g, p, x);
        if (g.side == IIM_SIDE_INTERIOR) return s < 0 ? K_PLUS : K_INACTIVE;
        if (g.side == IIM_SIDE_EXTERIOR) return s > 0 ? K_PLUS : K_INACTIVE;
        return s <= 0 ? K_MINUS : K_PLUS;
    }
    for (int d = 0; d < DIM; ++d) {
        x[d] = node_coord(g, ijk[d]);
        if (ijk[d] == 0 || ijk[d] == g.n) face = true;
    }
    int s = geom_sign_d<DIM>(g, p, x);
    if (face) {
        if (s <= 0) return 255;  // body touches the box
        return g.side == IIM_SIDE_INTERIOR ? K_INACTIVE : K_BOX;
    }
    if (g.side == IIM_SIDE_INTERIOR) return s < 0 ? K_PLUS : K_INACTIVE;
    if (g.side == IIM_SIDE_EXTERIOR) return s > 0 ? K_PLUS : K_INACTIVE;
    return s <= 0 ? K_MINUS : K_PLUS;
}

// Root of phi on the segment from node xa (coordinate vector) to xa + dir h e_axis.
// xa is the unknown for boundary problems, the Omega^- node for interfaces.
// Returns the coordinate along the axis, clamped to the segment; *which = sphere index.
__device__ inline double crossing_root(const Geom& g, const double* xa, int axis, int dir, int* which) {
#pragma clang fp contract(off)
    *which = 0;
    double a0 = xa[axis];
    double a1 = xa[axis] + (double)dir * g.h;
    double lo = fmin(a0, a1), hi = fmax(a0, a1);
    double root;
    if (g.kind == IIM_GEOM_SPHERE) {
        const double* c = g.p;
        double r = g.p[g.dim];
        double q = r * r;
        for (int o = 0; o < g.dim; ++o)
            if (o != axis) {
                double t = xa[o] - c[o];
                q = q - t * t;
            }
        double s = sqrt(fmax(q, 0.0));
        bool inside = (g.side != IIM_SIDE_EXTERIOR);  // interior problems and interfaces walk out
        root = inside ? c[axis] + (double)dir * s : c[axis] - (double)dir * s;
    } else if (g.kind == IIM_GEOM_GYROID) {
        // bisection (64 halvings) on the sign of phi; a zero at an end point is the root
        double lo_pt[3] = {xa[0], xa[1], xa[2]};
        if (dir < 0) lo_pt[axis] = xa[axis] - g.h;
        double hi_pt[3] = {lo_pt[0], lo_pt[1], lo_pt[2]};
        hi_pt[axis] = lo_pt[axis] + g.h;
        const int s_lo = sgn(gyroid_phi(g.p, lo_pt)), s_hi = sgn(gyroid_phi(g.p, hi_pt));
        if (s_lo == 0) {
            root = lo_pt[axis];
        } else if (s_hi == 0) {
            root = hi_pt[axis];
        } else {
            double a = lo_pt[axis], b = hi_pt[axis];
            double pt[3] = {lo_pt[0], lo_pt[1], lo_pt[2]};
            bool hit = false;
            root = 0.0;
            for (int it = 0; it < 64; ++it) {
                const double m = 0.5 * (a + b);
                pt[axis] = m;
                const int s = sgn(gyroid_phi(g.p, pt));
                if (s == 0) {
                    root = m;
                    hit = true;
                    break;
                }
                if (s == s_lo) a = m; else b = m;
            }
            if (!hit) root = 0.5 * (a + b);
        }
    } else if (g.kind == IIM_GEOM_STAR2D) {
        double lo_pt[2] = {xa[0], xa[1]};
        if (dir < 0) lo_pt[axis] = xa[axis] - g.h;
        double hi_pt[2] = {lo_pt[0], lo_pt[1]};
        hi_pt[axis] = lo_pt[axis] + g.h;
        int s_lo = sgn(star_phi(g.p, lo_pt[0], lo_pt[1]));
        int s_hi = sgn(star_phi(g.p, hi_pt[0], hi_pt[1]));
        if (s_lo == 0) {
            root = lo_pt[axis];
        } else if (s_hi == 0) {
            root = hi_pt[axis];
        } else {
            double a = lo_pt[axis], b = hi_pt[axis];
            double pt[2] = {lo_pt[0], lo_pt[1]};
            root = 0.0;
            bool hit = false;
            for (int it = 0; it < 64; ++it) {
                double m = 0.5 * (a + b);
                pt[axis] = m;
                int s = sgn(star_phi(g.p, pt[0], pt[1]));
                if (s == 0) {
                    root = m;
                    hit = true;
                    break;
                }
                if (s == s_lo) a = m; else b = m;
            }
            if (!hit) root = 0.5 * (a + b);
        }
    } else {
        int cnt = (int)llround(g.p[0]);
        double best = 0.0, best_x = a0;
        int best_i = -1;
        for (int s = 0; s < cnt; ++s) {
            const double* c = g.p + 1 + (g.dim + 1) * s;
            double r = c[g.dim];
            double q = r * r;
            for (int o = 0; o < g.dim; ++o)
                if (o != axis) {
                    double t = xa[o] - c[o];
                    q = q - t * t;
                }
            if (q < 0.0) continue;
            double sq = sqrt(q);
            double c0 = c[axis] - sq, c1 = c[axis] + sq;
            if (c1 < lo || c0 > hi) continue;
            double entry = dir > 0 ? c0 : c1;
            double dist = (entry - a0) * (double)dir;
            if (best_i < 0 || dist < best) {
                best = dist;
                best_i = s;
                best_x = entry;
            }
        }
        *which = best_i < 0 ? 0 : best_i;
        root = best_x;
    }
    return fmin(fmax(root, lo), hi);
}

// unit normal from Omega^- into Omega^+ at a point of Gamma
__device__ inline void geom_normal(const Geom& g, const double* x, int which, double* n) {
    double v[3] = {0.0, 0.0, 0.0};
    if (g.kind == IIM_GEOM_GYROID) {
        gyroid_grad(g.p, x, v);
    } else if (g.kind == IIM_GEOM_STAR2D) {
        double dx = x[0] - g.p[0], dy = x[1] - g.p[1];
        double rho = sqrt(dx * dx + dy * dy);
        double c = dx / rho;
        double T, U;
        cheb_tu((int)llround(g.p[4]), c, &T, &U);
        double dT = g.p[4] * U;
        double r3 = rho * rho * rho;
        v[0] = dx / rho - g.p[3] * dT * (dy * dy / r3);
        v[1] = dy / rho - g.p[3] * dT * (-dx * dy / r3);
    } else {
        const double* c = (g.kind == IIM_GEOM_SPHERE) ? g.p : g.p + 1 + (g.dim + 1) * which;
        for (int d = 0; d < g.dim; ++d) v[d] = x[d] - c[d];
    }
    double nn = 0.0;
    for (int d = 0; d < g.dim; ++d) nn += v[d] * v[d];
    nn = sqrt(nn);
    double sgn_ = (g.side == IIM_SIDE_INTERIOR) ? -1.0 : 1.0;
    for (int d = 0; d < 3; ++d) n[d] = d < g.dim ? sgn_ * v[d] / nn : 0.0;
}

// largest principal curvature magnitude at a point of Gamma
__device__ inline double geom_curvature(const Geom& g, const double* x, int which) {
    if (g.kind == IIM_GEOM_SPHERE) return 1.0 / g.p[g.dim];
    if (g.kind == IIM_GEOM_GYROID) return gyroid_curvature(g.p, x);
    if (g.kind == IIM_GEOM_SPHERE_UNION) return 1.0 / g.p[1 + (g.dim + 1) * which + g.dim];
    double dx = x[0] - g.p[0], dy = x[1] - g.p[1];
    double rho = sqrt(dx * dx + dy * dy);
    double c = dx / rho, s = dy / rho;
    double T, U;
    int L = (int)llround(g.p[4]);
    cheb_tu(L, c, &T, &U);
    double R = g.p[2] + g.p[3] * T;
    double Rp = -g.p[3] * L * s * U;
    double Rpp = -g.p[3] * L * L * T;
    return fabs(R * R + 2 * Rp * Rp - R * Rpp) / pow(R * R + Rp * Rp, 1.5);
}

// ---------------------------------------------------------------------------
// irregular high-order stencil slots (one int32 per axis direction)
// ---------------------------------------------------------------------------
enum : int { SLOT_REG = 0, SLOT_GHOST = 1, SLOT_BOX = 2 };
__host__ __device__ inline int slot_type(int s) { return s & 3; }
__host__ __device__ inline int slot_j(int s) { return (s >> 2) & 3; }
__host__ __device__ inline int slot_cs(int s) { return s >> 4; }
__host__ __device__ inline int make_slot(int type, int j, int cs) { return type | (j << 2) | (cs << 4); }

// 4th-order central second-derivative coefficients a_0, a_1, a_2
constexpr double A0 = -2.5, A1 = 4.0 / 3.0, A2 = -1.0 / 12.0;

// central second-derivative coefficient a_j of order 2W (W = 2: 4th order,
// W = 3: 6th order)
template <int W>
__host__ __device__ constexpr double ho_a(int j) {
    return W == 2 ? (j == 0 ? -2.5 : j == 1 ? 4.0 / 3.0 : -1.0 / 12.0)
                  : (j == 0 ? -49.0 / 18.0 : j == 1 ? 1.5 : j == 2 ? -3.0 / 20.0 : 1.0 / 90.0);
}

// central first derivative of order 2W (half-width W): du/dx ~ sum_j g_j
// (u_{+j} - u_{-j}) / h, j = 1..W (the gradient post-processing)
template <int W>
__host__ __device__ constexpr double ho_g(int j) {
    return W == 2 ? (j == 1 ? 2.0 / 3.0 : -1.0 / 12.0) : (j == 1 ? 0.75 : j == 2 ? -3.0 / 20.0 : 1.0 / 60.0);
}

// Lagrange weight of point t (t = 0 the box face, t = 1 .. 2W the nodes behind
// it) of the degree-2W polynomial through them, evaluated s steps beyond the face
template <int W>
__host__ __device__ constexpr double ho_ext(int s, int t) {
    constexpr double e2[5] = {5, -10, 10, -5, 1};
    constexpr double e31[7] = {7, -21, 35, -35, 21, -7, 1};
    constexpr double e32[7] = {28, -112, 210, -224, 140, -48, 7};
    return W == 2 ? e2[t] : (s == 1 ? e31[t] : e32[t]);
}

// ---------------------------------------------------------------------------
// wavefront reductions
// ---------------------------------------------------------------------------
// Wavefront sum on the VALU: DPP moves of the two 32-bit halves (quad
// permutes, row rotations, then the row broadcasts that gather the four
// 16-lane rows into lane 63), read back from lane 63.  All 64 lanes must be
// active.  The order of the additions is fixed, so the result is deterministic.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_copy(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// value of lane `lane` (wavefront-uniform) in every lane
__device__ inline double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ inline double wave_sum_valu(double v) {
    v += dpp_copy<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_copy<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_copy<0x124, 0xf>(v);  // row_ror 4
    v += dpp_copy<0x128, 0xf>(v);  // row_ror 8: every lane holds its row's sum
    v += dpp_copy<0x142, 0xa>(v);  // row_bcast 15 into rows 1 and 3
    v += dpp_copy<0x143, 0xc>(v);  // row_bcast 31 into rows 2 and 3
    return lane_value(v, 63);
}
// the same for the maximum of non-negative values (lanes outside a row mask read 0)
__device__ inline double wave_max_valu(double v) {
    v = fmax(v, dpp_copy<0xB1, 0xf>(v));
    v = fmax(v, dpp_copy<0x4E, 0xf>(v));
    v = fmax(v, dpp_copy<0x124, 0xf>(v));
    v = fmax(v, dpp_copy<0x128, 0xf>(v));
    v = fmax(v, dpp_copy<0x142, 0xa>(v));
    v = fmax(v, dpp_copy<0x143, 0xc>(v));
    return lane_value(v, 63);
}


inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace iim
