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

// half kicks of the levels lmin .. nlev-1, `times` times over (a closing and an opening kick)
__global__ void k_hier_kick(int n, const double* __restrict__ m, double* __restrict__ vx, double* __restrict__ vy,
                            double* __restrict__ vz, double* __restrict__ E, const double* __restrict__ lev, int lmin,
                            int nlev, double T, int times) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long nn = n;
    const double mi = m[i];
    double v[3] = {vx[i], vy[i], vz[i]};
    double e = E[i];
    for (int t = 0; t < times; t++)
        for (int l = lmin; l < nlev; l++) {
            const double dt = T / (double)(1ll << l);
            for (int c = 0; c < 3; c++) v[c] = v[c] + 0.5 * dt * lev[((long long)l * 4 + c) * nn + i] / mi;
            e = e + 0.5 * dt * lev[((long long)l * 4 + 3) * nn + i];
        }
    vx[i] = v[0];
    vy[i] = v[1];
    vz[i] = v[2];
    E[i] = e;
}

// drift by dt with the current velocity, wrapped into the box
__global__ void k_hier_drift(PassArrays a, Phys ph, double dt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double v[3] = {a.vx[i], a.vy[i], a.vz[i]};
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
}

// predicted velocity and u for the pass: the due levels' kicks with their previous rates
__global__ void k_hier_predict(int n, const double* __restrict__ m, const double* __restrict__ vx,
                               const double* __restrict__ vy, const double* __restrict__ vz,
                               const double* __restrict__ E, const double* __restrict__ lev, int lmin, int nlev,
                               double T, double u_floor, double* __restrict__ vp, double* __restrict__ up) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long nn = n;
    const double mi = m[i];
    double q[3] = {vx[i], vy[i], vz[i]};
    double Ep = E[i];
    for (int l = lmin; l < nlev; l++) {
        const double dt = T / (double)(1ll << l);
        for (int c = 0; c < 3; c++) q[c] = q[c] + 0.5 * dt * lev[((long long)l * 4 + c) * nn + i] / mi;
        Ep = Ep + 0.5 * dt * lev[((long long)l * 4 + 3) * nn + i];
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
                      int lmin, int nlev, double T, int times, hipStream_t s) {
    k_hier_kick<<<(n + 255) / 256, 256, 0, s>>>(n, m, vx, vy, vz, E, lev, lmin, nlev, T, times);
}

void launch_hier_drift(const PassArrays& a, const Phys& ph, double dt, hipStream_t s) {
    k_hier_drift<<<(a.n + 255) / 256, 256, 0, s>>>(a, ph, dt);
}

void launch_hier_predict(int n, const double* m, const double* vx, const double* vy, const double* vz,
                         const double* E, const double* lev, int lmin, int nlev, double T, double u_floor,
                         double* vp, double* up, hipStream_t s) {
    k_hier_predict<<<(n + 255) / 256, 256, 0, s>>>(n, m, vx, vy, vz, E, lev, lmin, nlev, T, u_floor, vp, up);
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
