// Kick-drift-kick update of the gas (MFM and MFV forms) and the Courant time-step reduction.
#include <math.h>

#include "device.h"
#include "kernels.h"

namespace mfm {

// first half kick (momentum and total energy), drift with the half-step
// velocity and wrap, predicted velocity and energy for the flux pass
__global__ void k_kick_drift(PassArrays a, Phys ph, double dt, double u_floor, double* __restrict__ vp,
                             double* __restrict__ up, double* __restrict__ Ehalf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const long long n = a.n;
    const double m = a.m[i];
    double v[3] = {a.vx[i], a.vy[i], a.vz[i]};
    double E = m * (a.u[i] + 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    for (int c = 0; c < 3; c++) v[c] = v[c] + 0.5 * dt * a.dp[c * n + i] / m;
    E = E + 0.5 * dt * a.dE[i];
    double* xs[3] = {(double*)a.x, (double*)a.y, (double*)a.z};
    for (int c = 0; c < 3; c++) {
        double xc = xs[c][i] + dt * v[c];
        if (ph.periodic[c]) {
            const double L = ph.box[c];
            xc = xc - L * floor(xc / L);
            if (xc >= L) xc = 0.0;
        }
        xs[c][i] = xc;
    }
    double q[3];
    for (int c = 0; c < 3; c++) q[c] = v[c] + 0.5 * dt * a.dp[c * n + i] / m;
    const double Ep = E + 0.5 * dt * a.dE[i];
    double uu = Ep / m - 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    uu = fmax(uu, u_floor);
    ((double*)a.vx)[i] = v[0];
    ((double*)a.vy)[i] = v[1];
    ((double*)a.vz)[i] = v[2];
    vp[i] = q[0];
    vp[n + i] = q[1];
    vp[2 * n + i] = q[2];
    up[i] = uu;
    Ehalf[i] = E;
}

// second half kick and recovery of u = E/m - |v|^2/2, floored
__global__ void k_kick2(PassArrays a, double dt, double u_floor, const double* __restrict__ Ehalf,
                        double* __restrict__ u, Counters* cnt) {
    cnt = counter_copy(cnt);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long fl = 0;
    if (i < a.n) {
        const long long n = a.n;
        const double m = a.m[i];
        double v[3] = {a.vx[i], a.vy[i], a.vz[i]};
        for (int c = 0; c < 3; c++) v[c] = v[c] + 0.5 * dt * a.dp[c * n + i] / m;
        const double E = Ehalf[i] + 0.5 * dt * a.dE[i];
        double uu = E / m - 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (uu < u_floor) {
            uu = u_floor;
            fl = 1;
        }
        ((double*)a.vx)[i] = v[0];
        ((double*)a.vy)[i] = v[1];
        ((double*)a.vz)[i] = v[2];
        u[i] = uu;
    }
    unsigned long long s = fl;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&cnt->floors, s);
}

// Finite-volume form: mass, momentum m v and total energy are kicked as
// conserved quantities with (dm, dp, dE), and v and u are recovered from them.
// First half kick, drift with the half-step velocity and wrap, and the
// predicted mass, velocity and u for the flux pass.  The half-step mass and
// velocity replace m and v; the half-step energy goes to Ehalf.
__global__ void k_kick_drift_mfv(PassArrays a, Phys ph, double dt, double u_floor, double* __restrict__ vp,
                                 double* __restrict__ up, double* __restrict__ Ehalf, double* __restrict__ mp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const long long n = a.n;
    const double m = a.m[i];
    const double v0[3] = {a.vx[i], a.vy[i], a.vz[i]};
    const double hdt = 0.5 * dt;
    const double mh = m + hdt * a.dm[i];
    double Qp[3], vh[3];
    for (int c = 0; c < 3; c++) {
        Qp[c] = m * v0[c] + hdt * a.dp[c * n + i];
        vh[c] = Qp[c] / mh;
    }
    const double Eh = m * (a.u[i] + 0.5 * (v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2])) + hdt * a.dE[i];
    double* xs[3] = {(double*)a.x, (double*)a.y, (double*)a.z};
    for (int c = 0; c < 3; c++) {
        double xc = xs[c][i] + dt * vh[c];
        if (ph.periodic[c]) {
            const double L = ph.box[c];
            xc = xc - L * floor(xc / L);
            if (xc >= L) xc = 0.0;
        }
        xs[c][i] = xc;
    }
    const double mq = mh + hdt * a.dm[i];
    double q[3];
    for (int c = 0; c < 3; c++) q[c] = (Qp[c] + hdt * a.dp[c * n + i]) / mq;
    double uu = (Eh + hdt * a.dE[i]) / mq - 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    uu = fmax(uu, u_floor);
    ((double*)a.m)[i] = mh;
    ((double*)a.vx)[i] = vh[0];
    ((double*)a.vy)[i] = vh[1];
    ((double*)a.vz)[i] = vh[2];
    vp[i] = q[0];
    vp[n + i] = q[1];
    vp[2 * n + i] = q[2];
    up[i] = uu;
    Ehalf[i] = Eh;
    mp[i] = mq;
}

// second half kick of the conserved quantities, then v = (m v)/m and
// u = E/m - |v|^2/2, floored
__global__ void k_kick2_mfv(PassArrays a, double dt, double u_floor, const double* __restrict__ Ehalf,
                            double* __restrict__ u, Counters* cnt) {
    cnt = counter_copy(cnt);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long fl = 0;
    if (i < a.n) {
        const long long n = a.n;
        const double hdt = 0.5 * dt;
        const double mh = a.m[i];
        const double vh[3] = {a.vx[i], a.vy[i], a.vz[i]};
        const double m1 = mh + hdt * a.dm[i];
        double v[3];
        for (int c = 0; c < 3; c++) v[c] = (mh * vh[c] + hdt * a.dp[c * n + i]) / m1;
        const double E = Ehalf[i] + hdt * a.dE[i];
        double uu = E / m1 - 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (uu < u_floor) {
            uu = u_floor;
            fl = 1;
        }
        ((double*)a.m)[i] = m1;
        ((double*)a.vx)[i] = v[0];
        ((double*)a.vy)[i] = v[1];
        ((double*)a.vz)[i] = v[2];
        u[i] = uu;
    }
    unsigned long long s = fl;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&cnt->floors, s);
}

// ------------------------------------------------------------ hierarchical steps
// The per-level rates of particle i sit at lev[(l * 4 + c) * n + i] (c: dp x, y,
// z, dE); level l steps by T / 2^l.  The expressions follow k_kick_drift and
// k_kick2 term by term, so with a single level the sequence of operations is
// the global step's.

// start of a step: total energy E = m (u + |v|^2/2), then the opening half kicks
// of every level (in registers, as k_kick_drift forms E and kicks it)
__global__ void k_hier_begin(int n, const double* __restrict__ m, double* __restrict__ vx, double* __restrict__ vy,
                             double* __restrict__ vz, const double* __restrict__ u, double* __restrict__ E,
                             const double* __restrict__ lev, int nlev, double T) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long nn = n;
    const double mi = m[i];
    double v[3] = {vx[i], vy[i], vz[i]};
    double e = mi * (u[i] + 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    for (int l = 0; l < nlev; l++) {
        const double dt = T / (double)(1ll << l);
        for (int c = 0; c < 3; c++) v[c] = v[c] + 0.5 * dt * lev[((long long)l * 4 + c) * nn + i] / mi;
        e = e + 0.5 * dt * lev[((long long)l * 4 + 3) * nn + i];
    }
    vx[i] = v[0];
    vy[i] = v[1];
    vz[i] = v[2];
    E[i] = e;
}

// half kicks of the levels lmin .. nlev-1, `times` times over (a closing and an
// opening kick); particle i's rates sit at column home[i] of lev
__global__ void k_hier_kick(int n, const double* __restrict__ m, double* __restrict__ vx, double* __restrict__ vy,
                            double* __restrict__ vz, double* __restrict__ E, const double* __restrict__ lev,
                            const long long* __restrict__ home, int lmin, int nlev, double T, int times) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long nn = n;
    const long long h = home[i];
    const double mi = m[i];
    double v[3] = {vx[i], vy[i], vz[i]};
    double e = E[i];
    for (int t = 0; t < times; t++)
        for (int l = lmin; l < nlev; l++) {
            const double dt = T / (double)(1ll << l);
            for (int c = 0; c < 3; c++) v[c] = v[c] + 0.5 * dt * lev[((long long)l * 4 + c) * nn + h] / mi;
            e = e + 0.5 * dt * lev[((long long)l * 4 + 3) * nn + h];
        }
    vx[i] = v[0];
    vy[i] = v[1];
    vz[i] = v[2];
    E[i] = e;
}

// drift by dt with the current velocity, wrapped into the box (with wrap);
// with moved, the path length since the last build accumulates per particle
// and its largest over the particles in moved[n]
__global__ void k_hier_drift(PassArrays a, Phys ph, double dt, int wrap, double* __restrict__ moved) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double path = 0.0;
    if (i < a.n) {
        const double v[3] = {a.vx[i], a.vy[i], a.vz[i]};
        double* xs[3] = {(double*)a.x, (double*)a.y, (double*)a.z};
        for (int c = 0; c < 3; c++) {
            double xc = xs[c][i] + dt * v[c];
            if (wrap && ph.periodic[c]) {
                const double L = ph.box[c];
                xc = xc - L * floor(xc / L);
                if (xc >= L) xc = 0.0;
            }
            xs[c][i] = xc;
        }
        if (moved) {
            path = moved[i] + fabs(dt) * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            moved[i] = path;
        }
    }
    if (moved) {
        // one atomic per wave whose largest path exceeds the largest seen so far
        // (a stale read only costs an atomic that changes nothing)
        for (int o = 32; o > 0; o >>= 1) path = fmax(path, __shfl_xor(path, o, kWave));
        unsigned long long* top = (unsigned long long*)(moved + a.n);
        const unsigned long long bits = (unsigned long long)__double_as_longlong(path);
        if ((threadIdx.x & (kWave - 1)) == 0 && bits > *(volatile unsigned long long*)top) atomicMax(top, bits);
    }
}

// predicted velocity and u for the pass: the due levels' kicks with their previous rates
__global__ void k_hier_predict(int n, const double* __restrict__ m, const double* __restrict__ vx,
                               const double* __restrict__ vy, const double* __restrict__ vz,
                               const double* __restrict__ E, const double* __restrict__ lev,
                               const long long* __restrict__ home, int lmin, int nlev, double T, double u_floor,
                               double* __restrict__ vp, double* __restrict__ up) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long nn = n;
    const long long h = home[i];
    const double mi = m[i];
    double q[3] = {vx[i], vy[i], vz[i]};
    double Ep = E[i];
    for (int l = lmin; l < nlev; l++) {
        const double dt = T / (double)(1ll << l);
        for (int c = 0; c < 3; c++) q[c] = q[c] + 0.5 * dt * lev[((long long)l * 4 + c) * nn + h] / mi;
        Ep = Ep + 0.5 * dt * lev[((long long)l * 4 + 3) * nn + h];
    }
    double uu = Ep / mi - 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    uu = fmax(uu, u_floor);
    vp[i] = q[0];
    vp[nn + i] = q[1];
    vp[2 * nn + i] = q[2];
    up[i] = uu;
}

// u = E/m - |v|^2/2 at the end of the step, floored (and counted)
__global__ void k_hier_finish(int n, const double* __restrict__ m, const double* __restrict__ vx,
                              const double* __restrict__ vy, const double* __restrict__ vz,
                              const double* __restrict__ E, double u_floor, double* __restrict__ u, Counters* cnt) {
    cnt = counter_copy(cnt);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long fl = 0;
    if (i < n) {
        const double v[3] = {vx[i], vy[i], vz[i]};
        double uu = E[i] / m[i] - 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (uu < u_floor) {
            uu = u_floor;
            fl = 1;
        }
        u[i] = uu;
    }
    unsigned long long s = fl;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&cnt->floors, s);
}

// min_i H_i / vsig_i: per-block partial minima, then one block over the partials
__global__ __launch_bounds__(256) void k_dt_partial(int n, const double* __restrict__ H,
                                                     const double* __restrict__ vsig, double* __restrict__ part) {
    __shared__ double sm[256];
    double v = INFINITY;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double t = H[i] / vsig[i];
        v = fmin(v, t);
    }
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_dt_final(int m, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sm[256];
    double v = INFINITY;
    for (int i = threadIdx.x; i < m; i += 256) v = fmin(v, part[i]);
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

int dt_min_parts(int n) {
    int b = (n + 255) / 256;
    return b < 1024 ? (b < 1 ? 1 : b) : 1024;
}

void launch_kick_drift(const PassArrays& a, const Phys& ph, double dt, double u_floor, double* vp, double* up,
                       double* Ehalf, hipStream_t s) {
    k_kick_drift<<<(a.n + 255) / 256, 256, 0, s>>>(a, ph, dt, u_floor, vp, up, Ehalf);
}

void launch_kick2(const PassArrays& a, double dt, double u_floor, const double* Ehalf, double* u, Counters* cnt,
                  hipStream_t s) {
    k_kick2<<<(a.n + 255) / 256, 256, 0, s>>>(a, dt, u_floor, Ehalf, u, cnt);
}

void launch_kick_drift_mfv(const PassArrays& a, const Phys& ph, double dt, double u_floor, double* vp, double* up,
                           double* Ehalf, double* mp, hipStream_t s) {
    k_kick_drift_mfv<<<(a.n + 255) / 256, 256, 0, s>>>(a, ph, dt, u_floor, vp, up, Ehalf, mp);
}

void launch_kick2_mfv(const PassArrays& a, double dt, double u_floor, const double* Ehalf, double* u,
                      Counters* cnt, hipStream_t s) {
    k_kick2_mfv<<<(a.n + 255) / 256, 256, 0, s>>>(a, dt, u_floor, Ehalf, u, cnt);
}

void launch_hier_begin(int n, const double* m, double* vx, double* vy, double* vz, const double* u, double* E,
                       const double* lev, int nlev, double T, hipStream_t s) {
    k_hier_begin<<<(n + 255) / 256, 256, 0, s>>>(n, m, vx, vy, vz, u, E, lev, nlev, T);
}

void launch_hier_kick(int n, const double* m, double* vx, double* vy, double* vz, double* E, const double* lev,
                      const long long* home, int lmin, int nlev, double T, int times, hipStream_t s) {
    k_hier_kick<<<(n + 255) / 256, 256, 0, s>>>(n, m, vx, vy, vz, E, lev, home, lmin, nlev, T, times);
}

__global__ void k_iota(int n, long long* __restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

void launch_iota(int n, long long* v, hipStream_t s) { k_iota<<<(n + 255) / 256, 256, 0, s>>>(n, v); }

void launch_hier_drift(const PassArrays& a, const Phys& ph, double dt, int wrap, double* moved, hipStream_t s) {
    k_hier_drift<<<(a.n + 255) / 256, 256, 0, s>>>(a, ph, dt, wrap, moved);
}

void launch_hier_predict(int n, const double* m, const double* vx, const double* vy, const double* vz,
                         const double* E, const double* lev, const long long* home, int lmin, int nlev, double T,
                         double u_floor, double* vp, double* up, hipStream_t s) {
    k_hier_predict<<<(n + 255) / 256, 256, 0, s>>>(n, m, vx, vy, vz, E, lev, home, lmin, nlev, T, u_floor, vp,
                                                   up);
}

// Whether the particles still stand where the last gradient pass packed them:
// *diff (zeroed by the caller) takes bit 1 when any position or kernel length
// differs bit for bit from the packed neighbour record (x, y, z, H).
__global__ void k_same_positions(int n, const double* __restrict__ x, const double* __restrict__ y,
                                 const double* __restrict__ z, const double* __restrict__ H,
                                 const double4* __restrict__ prim, unsigned long long* __restrict__ diff) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool d = false;
    if (i < n) {
        const double4 q = prim[4 * (long long)i];
        d = !(__double_as_longlong(q.x) == __double_as_longlong(x[i]) &&
              __double_as_longlong(q.y) == __double_as_longlong(y[i]) &&
              __double_as_longlong(q.z) == __double_as_longlong(z[i]) &&
              __double_as_longlong(q.w) == __double_as_longlong(H[i]));
    }
    if (__ballot(d) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(diff, 2ull);
}

void launch_same_positions(int n, const double* x, const double* y, const double* z, const double* H,
                           const double4* prim, unsigned long long* diff, hipStream_t s) {
    k_same_positions<<<(n + 255) / 256, 256, 0, s>>>(n, x, y, z, H, prim, diff);
}

// *bad |= 1 when some bin lies outside 0 .. max_bin
__global__ void k_check_bins(int n, const long long* __restrict__ bins, int max_bin,
                             unsigned long long* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool b = i < n && (bins[i] < 0 || bins[i] > max_bin);
    if (__ballot(b) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(bad, 1ull);
}

void launch_check_bins(int n, const long long* bins, int max_bin, unsigned long long* bad, hipStream_t s) {
    k_check_bins<<<(n + 255) / 256, 256, 0, s>>>(n, bins, max_bin, bad);
}

// One sweep of the neighbour time-step limiter: each bin raised to at least
// its flux neighbours' bins (as they stood before the sweep) minus one; the
// number raised is added to *raised.
__global__ void k_limit_bins(int n, int cap, const int* __restrict__ counts, const int* __restrict__ list,
                             const long long* __restrict__ bin, long long* __restrict__ out,
                             unsigned long long* __restrict__ raised) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool up = false;
    if (i < n) {
        const long long b = bin[i];
        long long nb = b;
        const int cnum = min(counts[i], cap);
        for (int k = 0; k < cnum; k++) nb = max(nb, bin[list[(long long)k * n + i]] - 1);
        out[i] = nb;
        up = nb != b;
    }
    const unsigned long long cnt = __popcll(__ballot(up));
    if (cnt && (threadIdx.x & (kWave - 1)) == 0) atomicAdd(raised, cnt);
}

void launch_limit_bins(int n, int cap, const int* counts, const int* list, const long long* bin, long long* out,
                       unsigned long long* raised, hipStream_t s) {
    k_limit_bins<<<(n + 255) / 256, 256, 0, s>>>(n, cap, counts, list, bin, out, raised);
}

// the flux lists back to their gather parts (counts = gcount), for a gradient
// pass that appends the tails again over the lists of an earlier solve
__global__ void k_reset_counts(int n, const int* __restrict__ gcount, int* __restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counts[i] = gcount[i];
}

void launch_reset_counts(int n, const int* gcount, int* counts, hipStream_t s) {
    k_reset_counts<<<(n + 255) / 256, 256, 0, s>>>(n, gcount, counts);
}

// ------------------------------------------- active subsets of hierarchical steps
// x wrapped into the box on periodic axes (positions between builds of a
// hierarchical step may stand just outside it)
__device__ __forceinline__ void wrap_box(const TreeDesc& td, const double x[3], double w[3]) {
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double v = x[d];
        if (td.periodic[d]) {
            v = v - td.box[d] * floor(v / td.box[d]);
            if (v >= td.box[d]) v = 0.0;
        }
        w[d] = v;
    }
}

// deposited key of the level-l cell holding x (x wrapped on periodic axes, per
// axis floor(x / side), clamped to the level's cells): the index of that
// cell's table entry past the level's offset
__device__ __forceinline__ unsigned long long cell_key(const TreeDesc& td, int l, const double x[3]) {
    unsigned long long key = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int c = min(td.ncell[l][d] - 1, max(0, (int)floor(x[d] / td.cs[l][d])));
        key |= deposit_bits((unsigned)c, td.mask[l][d]);
    }
    return key;
}

// A due particle marks its cell on every level.  Morton neighbours share their
// coarse cells, so within a wave only the first lane of a run of equal cells
// marks, and only when the bit is not already set.
__global__ void k_hier_mark(int n, const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, const long long* __restrict__ bins, int lmin, TreeDesc td,
                            unsigned* __restrict__ marks) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const bool act = i < n && bins[i] >= lmin;
    if (__ballot(act) == 0) return;   // uniform over the wave
    double xi[3] = {0.0, 0.0, 0.0};
    if (act) {
        const double xr[3] = {x[i], y[i], z[i]};
        wrap_box(td, xr, xi);
    }
    for (int l = 0; l <= td.bmax; l++) {
        const unsigned long long e = act ? (unsigned long long)td.tab_off[l] + cell_key(td, l, xi) : ~0ull;
        const unsigned lo = __shfl_up((unsigned)(e & 0xffffffffull), 1, kWave);
        const unsigned hi = __shfl_up((unsigned)(e >> 32), 1, kWave);
        const unsigned long long prev = ((unsigned long long)hi << 32) | lo;
        if (act && (lane == 0 || prev != e)) {
            const unsigned bit = 1u << (e & 31);
            if (!(marks[e >> 5] & bit)) atomicOr(&marks[e >> 5], bit);
        }
    }
}

// Every point within H of x (x wrapped into the box on periodic axes, as the
// marks are) lies in the 3x3x3 cells around x's cell on a level
// whose cells are at least H wide (per axis the cells c - 1 .. c + 1, wrapping
// on periodic axes of three or more cells; an axis of fewer cells is taken
// whole), and so does its cell by the same clamped floor; of those, only the
// cells whose box comes within H of x can hold it (on an open axis the edge
// cells reach out to infinity, as the clamp puts everything beyond them
// there).  A particle that is not due is kept with a gather list when one of
// them is marked.
__global__ void k_hier_mode(int n, const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, const double* __restrict__ H,
                            const long long* __restrict__ bins, int lmin, TreeDesc td,
                            const unsigned* __restrict__ marks, unsigned char* __restrict__ mode,
                            int* __restrict__ gcount, int* __restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (bins[i] >= lmin) {
        mode[i] = kModeSolve;
        return;
    }
    const double xr[3] = {x[i], y[i], z[i]};
    double xi[3];
    wrap_box(td, xr, xi);
    const double h = H[i];
    const double h2 = (h * (1.0 + 1e-9)) * (h * (1.0 + 1e-9));
    int l = td.bmax;
    while (l > 0 && fmin(td.cs[l][0], fmin(td.cs[l][1], td.cs[l][2])) < h) l--;
    int u0[3], cnt[3];
    unsigned long long dc[3], one[3];
    double g2[3][3];   // squared distance from x to the box of the o-th cell of the axis
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int nc = td.ncell[l][d];
        const double cs = td.cs[l][d];
        const int c = min(nc - 1, max(0, (int)floor(xi[d] / cs)));
        const unsigned long long m = td.mask[l][d];
        one[d] = m & (~m + 1);
        if (nc < 3) {
            u0[d] = 0;
            cnt[d] = nc;
            dc[d] = 0;
        } else if (td.periodic[d]) {
            u0[d] = c - 1;
            cnt[d] = 3;
            dc[d] = dilated_sub(deposit_bits((unsigned)c, m), one[d], m);
        } else {
            u0[d] = max(c - 1, 0);
            cnt[d] = min(c + 1, nc - 1) - u0[d] + 1;
            dc[d] = deposit_bits((unsigned)u0[d], m);
        }
#pragma unroll
        for (int o = 0; o < 3; o++) {
            const int u = u0[d] + o;   // unwrapped on periodic axes
            double lo = u * cs, hi = (u + 1) * cs;
            if (nc < 3) {
                lo = -INFINITY;
                hi = INFINITY;
            } else if (!td.periodic[d]) {
                if (u == 0) lo = -INFINITY;
                if (u == nc - 1) hi = INFINITY;
            }
            const double g = fmax(0.0, fmax(lo - xi[d], xi[d] - hi));
            g2[d][o] = g * g;
        }
    }
    const long long off = td.tab_off[l];
    bool hit = false;
    unsigned long long kx = dc[0];
    for (int ox = 0; ox < cnt[0] && !hit; ox++) {
        unsigned long long ky = dc[1];
        for (int oy = 0; oy < cnt[1] && !hit; oy++) {
            unsigned long long kz = dc[2];
            for (int oz = 0; oz < cnt[2] && !hit; oz++) {
                if (g2[0][ox] + g2[1][oy] + g2[2][oz] < h2) {
                    const unsigned long long e = (unsigned long long)off + (kx | ky | kz);
                    hit = (marks[e >> 5] >> (e & 31)) & 1u;
                }
                kz = dilated_add(kz, one[2], td.mask[l][2]);
            }
            ky = dilated_add(ky, one[1], td.mask[l][1]);
        }
        kx = dilated_add(kx, one[0], td.mask[l][0]);
    }
    mode[i] = hit ? kModeKept : kModeNone;
    if (!hit) {
        gcount[i] = 0;
        counts[i] = 0;
    }
}

void launch_hier_modes(int n, const double* x, const double* y, const double* z, const double* H,
                       const long long* bins, int lmin, const TreeDesc& td, long long tab_len, unsigned* marks,
                       unsigned char* mode, int* gcount, int* counts, hipStream_t s) {
    launch_fill_u64((tab_len + 63) / 64, (unsigned long long*)marks, 0ull, s);
    k_hier_mark<<<(n + 255) / 256, 256, 0, s>>>(n, x, y, z, bins, lmin, td, marks);
    k_hier_mode<<<(n + 255) / 256, 256, 0, s>>>(n, x, y, z, H, bins, lmin, td, marks, mode, gcount, counts);
}

void launch_hier_finish(int n, const double* m, const double* vx, const double* vy, const double* vz,
                        const double* E, double u_floor, double* u, Counters* cnt, hipStream_t s) {
    k_hier_finish<<<(n + 255) / 256, 256, 0, s>>>(n, m, vx, vy, vz, E, u_floor, u, cnt);
}

void launch_dt_min(int n, const double* H, const double* vsig, double* partial, int nparts, double* out,
                   hipStream_t s) {
    k_dt_partial<<<nparts, 256, 0, s>>>(n, H, vsig, partial);
    k_dt_final<<<1, 256, 0, s>>>(nparts, partial, out);
}

}  // namespace mfm
