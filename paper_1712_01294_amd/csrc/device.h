// Device-side building blocks of the gfx950 MFM pass: cubic-spline kernel,
// minimum-image displacement, and the stackless walk over the implicit octree
// that the Morton-sorted particle order and the per-level cell tables define.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfm {

constexpr int kMaxLevels = 12;   // levels 0..kMaxLevels-1
constexpr int kWave = 64;

// Everything a kernel needs to walk the cell tables, passed by value.
struct TreeDesc {
    int bmax;                        // deepest level
    int ktot;                        // key bits at bmax
    int leaf;                        // stop descending at <= leaf particles
    int nact[kMaxLevels];            // axes refined at level l (0 at l = 0)
    int actmask[kMaxLevels];         // bit d set when axis d refines at level l
    int kbits[kMaxLevels];           // key-prefix bits of a level-l cell
    long long tab_off[kMaxLevels];   // offset of level l in the (start, end) table
    double cs[kMaxLevels][3];        // cell side per axis at level l
    int ncell[kMaxLevels][3];        // cells per axis at level l (a power of two)
    unsigned long long mask[kMaxLevels][3];  // key-prefix bits of axis d at level l
    double box[3];
    int periodic[3];
    int qbits[3];                    // quantisation bits per axis
};

// Run-time physics parameters shared by the pass kernels.
struct Phys {
    double gamma;
    double n_ngb;
    double beta;
    double cond_max;
    double box[3];
    int periodic[3];
    int h_maxit;
    int max_ngb;
};

// Device counters (all updated with atomics, read by the host after a sync).
struct Counters {
    unsigned long long list_entries;
    unsigned long long list_max;
    unsigned long long h_iters;
    unsigned long long h_iters_max;
    unsigned long long noconv;
    unsigned long long minimage;
    unsigned long long overflow;
    unsigned long long illcond;
    unsigned long long fallbacks;
    unsigned long long clamps;
    unsigned long long nonfinite;
    unsigned long long floors;
    unsigned long long first_bad;    // min index (init ~0ull)
    unsigned long long cond_bits;    // max of the positive double cond, as bits
    unsigned long long h_rounds_max; // most group scans a kernel-length solve needed
    unsigned long long h_fallback;   // particles solved by the per-particle kernel
};

// ---------------------------------------------------------------- kernel
// Cubic spline with support radius H: W = 8/(pi H^3) w(q), q = r/H,
// w = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (1/2 < q <= 1), 0 beyond.
template <typename T>
__device__ __forceinline__ T spline_w(T q) {
    if (q <= T(0.5)) return T(1) + q * q * (T(6) * q - T(6));
    if (q <= T(1)) {
        T t = T(1) - q;
        return T(2) * t * t * t;
    }
    return T(0);
}

// q * dw/dq
template <typename T>
__device__ __forceinline__ T spline_qdw(T q) {
    if (q <= T(0.5)) return q * q * (T(18) * q - T(12));
    if (q <= T(1)) {
        T t = T(1) - q;
        return T(-6) * q * t * t;
    }
    return T(0);
}

template <typename T>
__device__ __forceinline__ T kernel_norm(T H) {
    return T(2.5464790894703255) / (H * H * H);  // 8/pi / H^3
}

// x_j - x_i on one axis, moved to the nearest periodic image
__device__ __forceinline__ double min_image(double d, double L, int periodic) {
    if (periodic) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

// distance along one axis from coordinate x to the interval [lo, hi)
__device__ __forceinline__ double axis_gap(double x, double lo, double hi, double L, int periodic) {
    if (x >= lo && x < hi) return 0.0;
    if (!periodic) return fmax(lo - x, x - hi);
    double g1 = lo - x;
    if (g1 < 0.0) g1 += L;
    double g2 = x - hi;
    if (g2 < 0.0) g2 += L;
    return fmin(g1, g2);
}

// ------------------------------------------------------ implicit octree walk
// Node = (level l, key prefix c, integer cell coordinates cx, cy, cz).
// A level-l cell holds the particles whose key starts with c: the sorted
// range tab[l][c] = [start, end).  `accept(l, c, cell_lo[3], cell_hi[3])`
// decides whether a non-empty node can hold a neighbour; `leaf(start, end)`
// scans a node's particles.  The walk visits nodes in Morton order without a
// stack: after a node it moves to the next sibling, climbing while the node
// is the last child of its parent.
template <typename Accept, typename Leaf>
__device__ __forceinline__ void tree_walk(const TreeDesc& td, const int2* __restrict__ tab,
                                          Accept&& accept, Leaf&& leaf) {
    int l = 0;
    unsigned long long c = 0;
    int cc[3] = {0, 0, 0};
    for (;;) {
        int2 se = tab[td.tab_off[l] + (long long)c];
        if (se.y > se.x) {
            double lo[3], hi[3];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                lo[d] = cc[d] * td.cs[l][d];
                hi[d] = lo[d] + td.cs[l][d];
            }
            if (accept(l, c, lo, hi)) {
                if (l == td.bmax || se.y - se.x <= td.leaf) {
                    leaf(se.x, se.y);
                } else {
                    // first child
                    l++;
                    int nb = td.nact[l];
                    c <<= nb;
                    int m = td.actmask[l];
#pragma unroll
                    for (int d = 0; d < 3; d++)
                        if (m & (1 << d)) cc[d] <<= 1;
                    continue;
                }
            }
        }
        // advance to the next sibling, climbing past last children
        for (;;) {
            if (l == 0) return;
            int nb = td.nact[l];
            unsigned k = (unsigned)(c & ((1ull << nb) - 1));
            if (k + 1 < (1u << nb)) {
                c++;
                k++;
                int m = td.actmask[l];
                int pos = nb;
#pragma unroll
                for (int d = 0; d < 3; d++)
                    if (m & (1 << d)) {
                        pos--;
                        cc[d] = (cc[d] & ~1) | ((k >> pos) & 1);
                    }
                break;
            }
            c >>= nb;
            int m = td.actmask[l];
#pragma unroll
            for (int d = 0; d < 3; d++)
                if (m & (1 << d)) cc[d] >>= 1;
            l--;
        }
    }
}

// squared distance from a point to a node box, with a relative pad so that a
// particle binned into a cell by rounding is never rejected by its bounds
__device__ __forceinline__ double node_dist2(const TreeDesc& td, const double xi[3],
                                             const double lo[3], const double hi[3]) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double pad = 1e-12 * td.box[d];
        double g = axis_gap(xi[d], lo[d] - pad, hi[d] + pad, td.box[d], td.periodic[d]);
        s += g * g;
    }
    return s;
}

// squared distance between a node box and a group box (both inside [0, box)),
// nearest periodic image per axis, padded like node_dist2
__device__ __forceinline__ double box_dist2(const TreeDesc& td, const double glo[3], const double ghi[3],
                                            const double lo[3], const double hi[3]) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double pad = 1e-12 * td.box[d];
        const double a = lo[d] - pad, b = hi[d] + pad;
        double g = fmax(0.0, fmax(a - ghi[d], glo[d] - b));
        if (td.periodic[d]) {
            const double L = td.box[d];
            g = fmin(g, fmax(0.0, fmax(a + L - ghi[d], glo[d] - b - L)));
            g = fmin(g, fmax(0.0, fmax(a - L - ghi[d], glo[d] - b + L)));
        }
        s += g * g;
    }
    return s;
}

// ------------------------------------------------------- cell stencil scan
// Each particle scans, on its own, the cells of one table level that overlap
// the cube [x - R, x + R]: the finest level whose cells are at least
// kStencilScale R wide, so a scan touches about (2 / kStencilScale + 1)^3
// cells.  Lanes of a wave (Morton neighbours) run the same loop shape on
// nearby cells, so there is no tree-shaped divergence.  Cell keys are stepped
// with dilated-integer increments on the per-axis bit masks of the key; on a
// periodic axis the increment past the last cell wraps to cell 0 by itself
// (cells per axis are a power of two).
constexpr double kStencilScale = 0.5;

// scatter the low bits of v into the set bits of mask (lowest first)
__device__ __forceinline__ unsigned long long deposit_bits(unsigned v, unsigned long long mask) {
    unsigned long long r = 0;
    while (mask) {
        const unsigned long long low = mask & (~mask + 1);
        if (v & 1u) r |= low;
        v >>= 1;
        mask &= mask - 1;
    }
    return r;
}

// key with the axis coordinate held in `mask` incremented by one
__device__ __forceinline__ unsigned long long dilated_inc(unsigned long long k, unsigned long long mask) {
    return (((k | ~mask) + 1) & mask) | (k & ~mask);
}

template <typename Visit>
__device__ __forceinline__ void stencil_scan(const TreeDesc& td, const int2* __restrict__ tab, const double xi[3],
                                             double R, Visit&& visit) {
    int L = td.bmax;
    while (L > 0 && fmin(td.cs[L][0], fmin(td.cs[L][1], td.cs[L][2])) < kStencilScale * R) L--;
    int lo[3], cnt[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double s = td.cs[L][d];
        const int nc = td.ncell[L][d];
        int a = (int)floor((xi[d] - R) / s);
        int b = (int)floor((xi[d] + R) / s);
        if (td.periodic[d]) {
            if (b - a + 1 >= nc) {
                a = 0;
                b = nc - 1;
            }
            cnt[d] = b - a + 1;
            a %= nc;
            if (a < 0) a += nc;
        } else {
            if (a < 0) a = 0;
            if (b > nc - 1) b = nc - 1;
            cnt[d] = b - a + 1;
        }
        lo[d] = a;
    }
    if (cnt[0] <= 0 || cnt[1] <= 0 || cnt[2] <= 0) return;
    const unsigned long long m0 = td.mask[L][0], m1 = td.mask[L][1], m2 = td.mask[L][2];
    const long long off = td.tab_off[L];
    unsigned long long kx = deposit_bits((unsigned)lo[0], m0) | deposit_bits((unsigned)lo[1], m1) |
                            deposit_bits((unsigned)lo[2], m2);
    for (int ix = 0; ix < cnt[0]; ix++) {
        unsigned long long ky = kx;
        for (int iy = 0; iy < cnt[1]; iy++) {
            unsigned long long kz = ky;
            for (int iz = 0; iz < cnt[2]; iz++) {
                const int2 se = tab[off + (long long)kz];
                for (int j = se.x; j < se.y; j++) visit(j);
                kz = dilated_inc(kz, m2);
            }
            ky = dilated_inc(ky, m1);
        }
        kx = dilated_inc(kx, m0);
    }
}

// wave-wide min / max of doubles (all 64 lanes participate)
__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace mfm
