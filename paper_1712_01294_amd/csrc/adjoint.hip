// Hand-written reverse mode of the MFM pass and of the kick-drift-kick step.
//
// The pass maps (x, v, u) to (dp/dt, dE/dt) through the kernel-length root
// H_i(x), the number density n_i, V_i = 1/n_i, rho = m n, P = (gamma-1) rho u,
// the gradient matrix E_i and B_i = E_i^-1, limited least-squares gradients,
// and per-pair faces, reconstruction and HLLC fluxes.  Its adjoint runs the
// stages backwards at fixed neighbour sets (the kernel is C^2 at its support
// edge, so set changes are smooth):
//   k_adj_pairs      each particle reverses the flux of every pair it is in
//                    (canonical order, as the forward) and keeps its own side,
//                    reading both sides from packed per-particle records;
//   k_adj_grad_*     reverse of limiter (active branch), E^-1, and the E / S
//                    sums, split into a per-particle part and a part that
//                    pulls the neighbour terms through the flux lists;
//   k_adj_length_*   reverse of n_i and V_i through W, and of H_i by the
//                    implicit-function theorem dH = -(dPhi/dx) / (dPhi/dH),
//                    split the same way.
// Min/max choices (Davis speeds, limiter, P* clamp, first-order fallback)
// follow the branch the forward took.
#include <math.h>

#include "device.h"
#include "kernels.h"

namespace mfm {

__device__ __forceinline__ int xcd_block_adj() {
    int G = gridDim.x, b = blockIdx.x;
    int x = b & 7, slot = b >> 3;
    int q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + slot;
}

__device__ __forceinline__ void disp(const Phys& ph, const double xi[3], double xj0, double xj1, double xj2,
                                     double d[3]) {
    d[0] = min_image(xj0 - xi[0], ph.box[0], ph.periodic[0]);
    d[1] = min_image(xj1 - xi[1], ph.box[1], ph.periodic[1]);
    d[2] = min_image(xj2 - xi[2], ph.box[2], ph.periodic[2]);
}

// W and its partial derivatives in r and H (cubic spline, support H)
__device__ __forceinline__ void kernel_wdw(double r, double H, double& W, double& dWdr, double& dWdH) {
    const double iH = 1.0 / H, q = r * iH, nrm = kernel_norm(H);
    const double w = spline_w(q);
    const double qdw = spline_qdw(q);
    W = nrm * w;
    dWdr = (q > 0.0) ? nrm * qdw / q * iH : 0.0;   // nrm w'(q) / H
    dWdH = -(3.0 * W + nrm * qdw) * iH;
}

// ----------------------------------------------------------- pair reverse
// Per-side data of one pair (FP64 record layout of the forward flux kernel)
struct Side {
    double H, V, phi[5], B[6], g[15];
};

struct SideAdj {
    double H, V, phi[5], B[6], g[15];
};

__device__ __forceinline__ void zero_adj(SideAdj& s) {
    s.H = s.V = 0.0;
#pragma unroll
    for (int k = 0; k < 5; k++) s.phi[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++) s.B[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 15; k++) s.g[k] = 0.0;
}

// y = B d for the symmetric B stored as xx xy xz yy yz zz
__device__ __forceinline__ void symv(const double B[6], const double d[3], double y[3]) {
    y[0] = B[0] * d[0] + B[1] * d[1] + B[2] * d[2];
    y[1] = B[1] * d[0] + B[3] * d[1] + B[4] * d[2];
    y[2] = B[2] * d[0] + B[4] * d[1] + B[5] * d[2];
}

// Reverse of one pair (left a, right b, d = x_b - x_a): given the adjoints of
// the momentum flux Fp (3) and energy flux FE, accumulate the adjoint of one
// side (a if own_a, else b) into lo, and the adjoint of d into ld.
__device__ __forceinline__ void pair_reverse(const Side& a, const Side& b, const double d[3], double gamma,
                                             const double lFp[3], double lFE, bool own_a, SideAdj& lo,
                                             double ld[3]) {
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double Wa, dWa_r, dWa_H, Wb, dWb_r, dWb_H;
    kernel_wdw(r, a.H, Wa, dWa_r, dWa_H);
    kernel_wdw(r, b.H, Wb, dWb_r, dWb_H);
    double ta[3], tb[3];
    symv(a.B, d, ta);
    symv(b.B, d, tb);
    const double ka = a.V * a.V * Wa, kb = b.V * b.V * Wb;
    double A[3];
    for (int c = 0; c < 3; c++) A[c] = ka * ta[c] + kb * tb[c];
    const double Amag = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
    if (!(Amag > 0.0)) return;
    const double nh[3] = {A[0] / Amag, A[1] / Amag, A[2] / Amag};
    const int slot_v = 1;
    double qL[5], qR[5];
    for (int f = 0; f < 5; f++) {
        const double* ga = a.g + 3 * f;
        const double* gb = b.g + 3 * f;
        qL[f] = a.phi[f] + 0.5 * (ga[0] * d[0] + ga[1] * d[1] + ga[2] * d[2]);
        qR[f] = b.phi[f] - 0.5 * (gb[0] * d[0] + gb[1] * d[1] + gb[2] * d[2]);
    }
    const bool fallback = !(qL[0] > 0.0) || !(qL[4] > 0.0) || !(qR[0] > 0.0) || !(qR[4] > 0.0);
    if (fallback)
        for (int f = 0; f < 5; f++) {
            qL[f] = a.phi[f];
            qR[f] = b.phi[f];
        }
    double w[3];
    for (int c = 0; c < 3; c++) w[c] = 0.5 * (a.phi[slot_v + c] + b.phi[slot_v + c]);
    double uL = 0.0, uR = 0.0;
    for (int c = 0; c < 3; c++) {
        uL += (qL[slot_v + c] - w[c]) * nh[c];
        uR += (qR[slot_v + c] - w[c]) * nh[c];
    }
    const double rL = qL[0], pL = qL[4], rR = qR[0], pR = qR[4];
    const double cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);
    const bool sl_left = (uL - cL < uR - cR);
    const double SL = sl_left ? uL - cL : uR - cR;
    const bool sr_left = (uL + cL > uR + cR);
    const double SR = sr_left ? uL + cL : uR + cR;
    const double mL = rL * (SL - uL), mR = rR * (SR - uR);
    const double num = pR - pL + mL * uL - mR * uR;
    const double den = mL - mR;
    const double Ss = num / den;
    double Ps = 0.5 * (pL + pR + mL * (Ss - uL) + mR * (Ss - uR));
    const bool clamped = Ps < 0.0;
    if (clamped) Ps = 0.0;
    const double wn = w[0] * nh[0] + w[1] * nh[1] + w[2] * nh[2];

    // ---- reverse sweep
    double lA[3], lnh[3] = {0, 0, 0}, lw[3] = {0, 0, 0};
    double lPs = 0.0;
    for (int c = 0; c < 3; c++) {
        lPs += lFp[c] * A[c];
        lA[c] = Ps * lFp[c];
    }
    lPs += lFE * (Ss + wn) * Amag;
    double lSs = lFE * Ps * Amag;
    const double lwn = lFE * Ps * Amag;
    double lAmag = lFE * Ps * (Ss + wn);
    for (int c = 0; c < 3; c++) {
        lw[c] += lwn * nh[c];
        lnh[c] += lwn * w[c];
    }
    if (clamped) lPs = 0.0;
    double lpL = 0.5 * lPs, lpR = 0.5 * lPs;
    double lmL = 0.5 * lPs * (Ss - uL), lmR = 0.5 * lPs * (Ss - uR);
    lSs += 0.5 * lPs * (mL + mR);
    double luL = -0.5 * lPs * mL, luR = -0.5 * lPs * mR;
    const double lnum = lSs / den;
    const double lden = -lSs * Ss / den;
    lmL += lden;
    lmR -= lden;
    lpR += lnum;
    lpL -= lnum;
    lmL += lnum * uL;
    luL += lnum * mL;
    lmR -= lnum * uR;
    luR -= lnum * mR;
    double lrL = lmL * (SL - uL), lrR = lmR * (SR - uR);
    const double lSL = lmL * rL, lSR = lmR * rR;
    luL -= lmL * rL;
    luR -= lmR * rR;
    double lcL = 0.0, lcR = 0.0;
    if (sl_left) {
        luL += lSL;
        lcL -= lSL;
    } else {
        luR += lSL;
        lcR -= lSL;
    }
    if (sr_left) {
        luL += lSR;
        lcL += lSR;
    } else {
        luR += lSR;
        lcR += lSR;
    }
    lpL += lcL * gamma / (2.0 * cL * rL);
    lrL -= lcL * cL / (2.0 * rL);
    lpR += lcR * gamma / (2.0 * cR * rR);
    lrR -= lcR * cR / (2.0 * rR);
    double lqL[5], lqR[5];
    lqL[0] = lrL;
    lqL[4] = lpL;
    lqR[0] = lrR;
    lqR[4] = lpR;
    for (int c = 0; c < 3; c++) {
        lqL[slot_v + c] = luL * nh[c];
        lqR[slot_v + c] = luR * nh[c];
        lw[c] -= (luL + luR) * nh[c];
        lnh[c] += luL * (qL[slot_v + c] - w[c]) + luR * (qR[slot_v + c] - w[c]);
    }
    for (int c = 0; c < 3; c++) lo.phi[slot_v + c] += 0.5 * lw[c];
    for (int f = 0; f < 5; f++) {
        lo.phi[f] += own_a ? lqL[f] : lqR[f];
        if (!fallback) {
            for (int k = 0; k < 3; k++) {
                lo.g[3 * f + k] += own_a ? 0.5 * lqL[f] * d[k] : -(0.5 * lqR[f] * d[k]);
                ld[k] += 0.5 * lqL[f] * a.g[3 * f + k];
                ld[k] -= 0.5 * lqR[f] * b.g[3 * f + k];
            }
        }
    }
    // n = A / |A|, |A|
    const double nl = nh[0] * lnh[0] + nh[1] * lnh[1] + nh[2] * lnh[2];
    for (int c = 0; c < 3; c++) lA[c] += (lnh[c] - nh[c] * nl) / Amag + lAmag * nh[c];
    // A = ka ta + kb tb
    double lta[3], ltb[3];
    double lka = 0.0, lkb = 0.0;
    for (int c = 0; c < 3; c++) {
        lka += lA[c] * ta[c];
        lkb += lA[c] * tb[c];
        lta[c] = lA[c] * ka;
        ltb[c] = lA[c] * kb;
    }
    // y = B d: the own side's B takes lt d^T (stored components), d takes B lt from both
    {
        const double* lt = own_a ? lta : ltb;
        lo.B[0] += lt[0] * d[0];
        lo.B[1] += lt[0] * d[1] + lt[1] * d[0];
        lo.B[2] += lt[0] * d[2] + lt[2] * d[0];
        lo.B[3] += lt[1] * d[1];
        lo.B[4] += lt[1] * d[2] + lt[2] * d[1];
        lo.B[5] += lt[2] * d[2];
        double t[3];
        symv(a.B, lta, t);
        for (int c = 0; c < 3; c++) ld[c] += t[c];
        symv(b.B, ltb, t);
        for (int c = 0; c < 3; c++) ld[c] += t[c];
    }
    const double lWa = lka * a.V * a.V, lWb = lkb * b.V * b.V;
    lo.V += own_a ? lka * 2.0 * a.V * Wa : lkb * 2.0 * b.V * Wb;
    const double lr = lWa * dWa_r + lWb * dWb_r;
    lo.H += own_a ? lWa * dWa_H : lWb * dWb_H;
    if (r > 0.0)
        for (int k = 0; k < 3; k++) ld[k] += lr * d[k] / r;
}

// Adjoint storage: acc_x (3n, atomic target), acc_phi (5n: rho, vx, vy, vz, P;
// atomic target), acc_H, acc_V (n), acc_B (6n), acc_g (15n).
struct AdjArrays {
    double *acc_x, *acc_phi, *acc_H, *acc_V, *acc_B, *acc_g;
};

// Side record of the pair reverse, one per particle (kAdjRec doubles, in the
// region the gradient reverse later fills with its own records): x, y, z, H,
// V, phi (5), B (6), grad (15), then the adjoints of dp (3) and dE it receives.
enum { S_X = 0, S_H = 3, S_V = 4, S_PHI = 5, S_B = 10, S_G = 16, S_LP = 31, S_LE = 34 };

__global__ void k_adj_side_pack(PassArrays a, const double* __restrict__ lam_dp, const double* __restrict__ lam_dE,
                                double* __restrict__ rec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const long long n = a.n;
    double* rc = rec + (long long)i * kAdjRec;
    rc[S_X] = a.x[i];
    rc[S_X + 1] = a.y[i];
    rc[S_X + 2] = a.z[i];
    rc[S_H] = a.H[i];
    rc[S_V] = a.V[i];
    rc[S_PHI] = a.rho[i];
    rc[S_PHI + 1] = a.vx[i];
    rc[S_PHI + 2] = a.vy[i];
    rc[S_PHI + 3] = a.vz[i];
    rc[S_PHI + 4] = a.P[i];
    for (int k = 0; k < 6; k++) rc[S_B + k] = a.B[k * n + i];
    for (int k = 0; k < 15; k++) rc[S_G + k] = a.grad[k * n + i];
    for (int c = 0; c < 3; c++) rc[S_LP + c] = lam_dp[c * n + i];
    rc[S_LE] = lam_dE[i];
}

__device__ __forceinline__ void side_of(const double* __restrict__ rc, Side& s) {
    s.H = rc[S_H];
    s.V = rc[S_V];
#pragma unroll
    for (int k = 0; k < 5; k++) s.phi[k] = rc[S_PHI + k];
#pragma unroll
    for (int k = 0; k < 6; k++) s.B[k] = rc[S_B + k];
#pragma unroll
    for (int k = 0; k < 15; k++) s.g[k] = rc[S_G + k];
}

// Each particle reverses the flux of every pair in its flux list (with the
// pair's canonical left/right order, as the forward) and keeps its own side.
// Both records are loaded per pair in left/right order (the own one stays in
// cache), so one inlined reverse serves both orders.
constexpr int kAdjPairWaves = 1;
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAdjPairWaves))) void k_adj_pairs(PassArrays a, Phys ph, const int* __restrict__ counts,
                                                    const int* __restrict__ list, const double* __restrict__ rec,
                                                    AdjArrays aj) {
    const int i = xcd_block_adj() * 256 + threadIdx.x;
    if (i >= a.n) return;
    const long long n = a.n;
    SideAdj own;
    zero_adj(own);
    double lx[3] = {0.0, 0.0, 0.0};
    const int cnum = counts[i];
    int jn = cnum > 0 ? list[i] : 0;   // the next list entry, loaded one neighbour ahead
    for (int k = 0; k < cnum; k++) {
        const int j = jn;
        if (k + 1 < cnum) jn = list[(long long)(k + 1) * n + i];
        const bool iL = i < j;
        const double* rL = rec + (long long)(iL ? i : j) * kAdjRec;
        const double* rR = rec + (long long)(iL ? j : i) * kAdjRec;
        Side sL, sR;
        side_of(rL, sL);
        side_of(rR, sR);
        // canonical displacement x_R - x_L as in the forward
        const double xL[3] = {rL[S_X], rL[S_X + 1], rL[S_X + 2]};
        double d[3];
        disp(ph, xL, rR[S_X], rR[S_X + 1], rR[S_X + 2], d);
        // dp_L -= Fp, dp_R += Fp
        double lFp[3];
        for (int c = 0; c < 3; c++) lFp[c] = rR[S_LP + c] - rL[S_LP + c];
        const double lFE = rR[S_LE] - rL[S_LE];
        double ld[3] = {0.0, 0.0, 0.0};
        pair_reverse(sL, sR, d, ph.gamma, lFp, lFE, iL, own, ld);
        // d = x_R - x_L
        const double sg = iL ? -1.0 : 1.0;
        for (int c = 0; c < 3; c++) lx[c] += sg * ld[c];
    }
    for (int c = 0; c < 3; c++) aj.acc_x[c * n + i] = lx[c];
    for (int f = 0; f < 5; f++) aj.acc_phi[f * n + i] = own.phi[f];
    aj.acc_H[i] = own.H;
    aj.acc_V[i] = own.V;
    for (int k = 0; k < 6; k++) aj.acc_B[k * n + i] = own.B[k];
    for (int k = 0; k < 15; k++) aj.acc_g[k * n + i] = own.g[k];
}

// ------------------------------------------------------- gradient reverse
// The gradient stage of particle i sums over its gather set (j with r_ij < H_i).
// Its reverse gives each such pair a term for i and a term for j.  Part one
// (one thread per i) rebuilds the sums, reverses the limiter, E^-1 and the
// sums, keeps the terms for i, and writes a record of what the terms for the
// neighbours need; part two (one thread per j) walks j's flux list, which holds
// every i whose gather set contains j, and adds the terms for j from the
// records.  No thread writes another particle's sums: the terms that i's
// limiter gives single neighbours (the farthest one, which sets its length, and
// the holders of each field's extrema) travel in i's record too, with those
// neighbours' indices, and part two adds them when it meets i.  Every sum is
// then taken in a fixed order and the reverse is bitwise deterministic.
//
// Record per particle (kRec doubles): x, y, z, H, V, phi (5), the adjoint of
// E as a full 3x3 matrix (9), the adjoints of the gradient sums S (15).  The
// limiter terms addressed to single neighbours sit in a block of their own, so
// that the records every pair reads stay small: 16 int32 indices per particle
// in one 64-byte line (the farthest neighbour, the holders of the 5 maxima and
// of the 5 minima; -1 where no term goes to a neighbour; 4 unused), read by
// every pair, and 12 values (the adjoint of the limiter length, the maxima's
// and the minima's terms; 1 unused), read only where an index matches.
constexpr int kRec = kAdjRec;
enum { P_X = 0, P_H = 3, P_V = 4, P_PHI = 5, P_LE = 10, P_LS = 19 };
static_assert(P_LS + 15 <= kRec, "record slots");
enum { L_HALF = 0, L_MAX = 1, L_MIN = 6 };
static_assert(kAdjLim * 2 >= 16 + 2 * 12, "limiter block");
// own-side adjoints of part one, read back by part two: phi (5), x (3)
static_assert(kAdjOwn == 8, "own-side slots");

struct PullArrays {
    double* rec;   // kRec x n, particle-major
    double* own;   // kOwn x n, field-major
    int* lix;      // 16 x n int32, particle-major
    double* lval;  // 12 x n, particle-major
};

// the term that pair (i -> j) of i's gather set gives j: adds to lphi (5) and
// ld (3, the adjoint of d = x_j - x_i); the same expression serves part one
__device__ __forceinline__ void grad_pair_terms(const double d[3], double r, double Hi, double Vi,
                                                const double* LE, const double* lS, const double dphi[5],
                                                double t[5], double ld[3], double& lpsi_out, double& W,
                                                double& dWH) {
    double dWr;
    kernel_wdw(r, Hi, W, dWr, dWH);
    const double psi = W * Vi;
    double Ld[3], LTd[3];
    for (int c = 0; c < 3; c++) {
        Ld[c] = LE[3 * c] * d[0] + LE[3 * c + 1] * d[1] + LE[3 * c + 2] * d[2];
        LTd[c] = LE[c] * d[0] + LE[3 + c] * d[1] + LE[6 + c] * d[2];
    }
    double lpsi = d[0] * Ld[0] + d[1] * Ld[1] + d[2] * Ld[2];
    for (int c = 0; c < 3; c++) ld[c] = (Ld[c] + LTd[c]) * psi;
    for (int f = 0; f < 5; f++) {
        const double* ls = lS + 3 * f;
        const double dl = d[0] * ls[0] + d[1] * ls[1] + d[2] * ls[2];
        lpsi += dphi[f] * dl;
        for (int c = 0; c < 3; c++) ld[c] += dphi[f] * psi * ls[c];
        t[f] = psi * dl;
    }
    const double lW = lpsi * Vi;
    if (r > 0.0)
        for (int c = 0; c < 3; c++) ld[c] += lW * dWr * d[c] / r;
    lpsi_out = lpsi;
}

__global__ __launch_bounds__(256) void k_adj_grad_own(PassArrays a, Phys ph, const int* __restrict__ gcount,
                                                       const int* __restrict__ list, AdjArrays aj, PullArrays pa) {
    const int i = xcd_block_adj() * 256 + threadIdx.x;
    if (i >= a.n) return;
    const long long n = a.n;
    const double xi[3] = {a.x[i], a.y[i], a.z[i]};
    const double Hi = a.H[i], Vi = a.V[i];
    const double rho_i = a.m[i] * a.nk[i];
    const double phi_i[5] = {rho_i, a.vx[i], a.vy[i], a.vz[i], (ph.gamma - 1.0) * rho_i * a.u[i]};
    const int cnum = gcount[i];
    // recompute the forward sums, extrema and their owners
    double E[6] = {0, 0, 0, 0, 0, 0}, S[15];
    for (int k = 0; k < 15; k++) S[k] = 0.0;
    double pmax[5], pmin[5];
    int jmax[5], jmin[5];
    for (int f = 0; f < 5; f++) {
        pmax[f] = pmin[f] = phi_i[f];
        jmax[f] = jmin[f] = i;
    }
    double rmax = 0.0;
    int jr = i;
    int jn = cnum > 0 ? list[i] : 0;   // the next list entry, loaded one neighbour ahead
    for (int k = 0; k < cnum; k++) {
        const int j = jn;
        if (k + 1 < cnum) jn = list[(long long)(k + 1) * n + i];
        double d[3];
        disp(ph, xi, a.x[j], a.y[j], a.z[j], d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double W, dWr, dWH;
        kernel_wdw(r, Hi, W, dWr, dWH);
        const double psi = W * Vi;
        const double rho_j = a.m[j] * a.nk[j];
        const double phi_j[5] = {rho_j, a.vx[j], a.vy[j], a.vz[j], (ph.gamma - 1.0) * rho_j * a.u[j]};
        E[0] += d[0] * d[0] * psi;
        E[1] += d[0] * d[1] * psi;
        E[2] += d[0] * d[2] * psi;
        E[3] += d[1] * d[1] * psi;
        E[4] += d[1] * d[2] * psi;
        E[5] += d[2] * d[2] * psi;
        for (int f = 0; f < 5; f++) {
            const double df = (phi_j[f] - phi_i[f]) * psi;
            S[3 * f] += df * d[0];
            S[3 * f + 1] += df * d[1];
            S[3 * f + 2] += df * d[2];
            if (phi_j[f] > pmax[f]) {
                pmax[f] = phi_j[f];
                jmax[f] = j;
            }
            if (phi_j[f] < pmin[f]) {
                pmin[f] = phi_j[f];
                jmin[f] = j;
            }
        }
        if (r > rmax) {
            rmax = r;
            jr = j;
        }
    }
    const double c00 = E[3] * E[5] - E[4] * E[4];
    const double c01 = E[2] * E[4] - E[1] * E[5];
    const double c02 = E[1] * E[4] - E[2] * E[3];
    const double c11 = E[0] * E[5] - E[2] * E[2];
    const double c12 = E[1] * E[2] - E[0] * E[4];
    const double c22 = E[0] * E[3] - E[1] * E[1];
    const double det = E[0] * c00 + E[1] * c01 + E[2] * c02;
    const double id = 1.0 / det;
    const double B[6] = {c00 * id, c01 * id, c02 * id, c11 * id, c12 * id, c22 * id};
    const double Bf[3][3] = {{B[0], B[1], B[2]}, {B[1], B[3], B[4]}, {B[2], B[4], B[5]}};
    const double half = 0.5 * rmax;
    // Lambda: full 3x3 adjoint of B; the stored-component adjoint of an
    // off-diagonal entry is split evenly between its two positions
    double Lam[3][3];
    {
        const double lb[6] = {aj.acc_B[0 * n + i], aj.acc_B[1 * n + i], aj.acc_B[2 * n + i],
                              aj.acc_B[3 * n + i], aj.acc_B[4 * n + i], aj.acc_B[5 * n + i]};
        Lam[0][0] = lb[0];
        Lam[1][1] = lb[3];
        Lam[2][2] = lb[5];
        Lam[0][1] = Lam[1][0] = 0.5 * lb[1];
        Lam[0][2] = Lam[2][0] = 0.5 * lb[2];
        Lam[1][2] = Lam[2][1] = 0.5 * lb[4];
    }
    double lS[15];
    double lphi_i[5] = {0, 0, 0, 0, 0};
    double lhalf = 0.0;
    double lmax[5], lmin[5];
    for (int f = 0; f < 5; f++) {
        const double* s = S + 3 * f;
        double g[3];
        for (int c = 0; c < 3; c++) g[c] = Bf[c][0] * s[0] + Bf[c][1] * s[1] + Bf[c][2] * s[2];
        const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        double alpha = 1.0, up = 0.0, dn = 0.0;
        if (gn > 0.0) {
            up = (pmax[f] - phi_i[f]) / (gn * half);
            dn = (phi_i[f] - pmin[f]) / (gn * half);
            alpha = fmin(1.0, ph.beta * fmin(up, dn));
        }
        double lg[3];
        double lalpha = 0.0;
        for (int c = 0; c < 3; c++) {
            const double lgr = aj.acc_g[(3 * f + c) * n + i];
            lg[c] = alpha * lgr;
            lalpha += lgr * g[c];
        }
        lmax[f] = lmin[f] = 0.0;
        if (gn > 0.0 && alpha < 1.0) {
            const double lm = ph.beta * lalpha;
            const double den = gn * half;
            double lgn = 0.0;
            if (up <= dn) {
                lmax[f] += lm / den;
                lphi_i[f] -= lm / den;
                lgn -= lm * up / gn;
                lhalf -= lm * up / half;
            } else {
                lphi_i[f] += lm / den;
                lmin[f] -= lm / den;
                lgn -= lm * dn / gn;
                lhalf -= lm * dn / half;
            }
            for (int c = 0; c < 3; c++) lg[c] += lgn * g[c] / gn;
        }
        // g = B s
        for (int c = 0; c < 3; c++)
            for (int q = 0; q < 3; q++) Lam[c][q] += lg[c] * s[q];
        for (int q = 0; q < 3; q++) lS[3 * f + q] = Bf[q][0] * lg[0] + Bf[q][1] * lg[1] + Bf[q][2] * lg[2];
    }
    // E^-1: lE = -B Lam B (row-major 3x3)
    double T[3][3], LE[9];
    for (int c = 0; c < 3; c++)
        for (int q = 0; q < 3; q++) T[c][q] = Lam[c][0] * Bf[0][q] + Lam[c][1] * Bf[1][q] + Lam[c][2] * Bf[2][q];
    for (int c = 0; c < 3; c++)
        for (int q = 0; q < 3; q++) LE[3 * c + q] = -(Bf[c][0] * T[0][q] + Bf[c][1] * T[1][q] + Bf[c][2] * T[2][q]);
    // record for the neighbours' part two
    double* rc = pa.rec + (long long)i * kRec;
    rc[P_X] = xi[0];
    rc[P_X + 1] = xi[1];
    rc[P_X + 2] = xi[2];
    rc[P_H] = Hi;
    rc[P_V] = Vi;
    for (int f = 0; f < 5; f++) rc[P_PHI + f] = phi_i[f];
    for (int k = 0; k < 9; k++) rc[P_LE + k] = LE[k];
    for (int k = 0; k < 15; k++) rc[P_LS + k] = lS[k];
    // i's side of every pair of its gather set
    double lH = 0.0, lV = 0.0;
    double lxi[3] = {0.0, 0.0, 0.0};
    jn = cnum > 0 ? list[i] : 0;   // the next list entry, loaded one neighbour ahead
    for (int k = 0; k < cnum; k++) {
        const int j = jn;
        if (k + 1 < cnum) jn = list[(long long)(k + 1) * n + i];
        double d[3];
        disp(ph, xi, a.x[j], a.y[j], a.z[j], d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double rho_j = a.m[j] * a.nk[j];
        const double dphi[5] = {rho_j - phi_i[0], a.vx[j] - phi_i[1], a.vy[j] - phi_i[2], a.vz[j] - phi_i[3],
                                (ph.gamma - 1.0) * rho_j * a.u[j] - phi_i[4]};
        double t[5], ld[3], lpsi, W, dWH;
        grad_pair_terms(d, r, Hi, Vi, LE, lS, dphi, t, ld, lpsi, W, dWH);
        lV += lpsi * W;
        lH += lpsi * Vi * dWH;
        for (int f = 0; f < 5; f++) lphi_i[f] -= t[f];
        for (int c = 0; c < 3; c++) lxi[c] -= ld[c];
        if (j == jr && r > 0.0)
            for (int c = 0; c < 3; c++) {
                // the farthest neighbour sets the limiter's length; its own term goes
                // through the record (part two adds the same th for j)
                const double th = 0.5 * lhalf * d[c] / r;
                lxi[c] -= th;
            }
    }
    int ix[16];
    double* lv = pa.lval + (long long)i * 12;
    ix[0] = jr != i ? jr : -1;
    lv[L_HALF] = lhalf;
    for (int f = 0; f < 5; f++) {
        int tmax = -1, tmin = -1;
        if (lmax[f] != 0.0) {
            if (jmax[f] == i) lphi_i[f] += lmax[f];
            else tmax = jmax[f];
        }
        if (lmin[f] != 0.0) {
            if (jmin[f] == i) lphi_i[f] += lmin[f];
            else tmin = jmin[f];
        }
        ix[1 + f] = tmax;
        ix[6 + f] = tmin;
        lv[L_MAX + f] = lmax[f];
        lv[L_MIN + f] = lmin[f];
    }
    for (int q = 11; q < 16; q++) ix[q] = -1;
    int4* ixo = (int4*)(pa.lix + (long long)i * 16);
    for (int q = 0; q < 4; q++) ixo[q] = make_int4(ix[4 * q], ix[4 * q + 1], ix[4 * q + 2], ix[4 * q + 3]);
    for (int f = 0; f < 5; f++) pa.own[f * n + i] = lphi_i[f];
    for (int c = 0; c < 3; c++) pa.own[(5 + c) * n + i] = lxi[c];
    aj.acc_H[i] += lH;
    aj.acc_V[i] += lV;
}

__global__ __launch_bounds__(256) void k_adj_grad_pull(PassArrays a, Phys ph, const int* __restrict__ counts,
                                                        const int* __restrict__ list, AdjArrays aj, PullArrays pa) {
    const int j = xcd_block_adj() * 256 + threadIdx.x;
    if (j >= a.n) return;
    const long long n = a.n;
    const double xj[3] = {a.x[j], a.y[j], a.z[j]};
    const double rho_j = a.m[j] * a.nk[j];
    const double phi_j[5] = {rho_j, a.vx[j], a.vy[j], a.vz[j], (ph.gamma - 1.0) * rho_j * a.u[j]};
    double lphi[5], lx[3];
    for (int f = 0; f < 5; f++) lphi[f] = pa.own[f * n + j];
    for (int c = 0; c < 3; c++) lx[c] = pa.own[(5 + c) * n + j];
    const int cnum = counts[j];
    for (int k = 0; k < cnum; k++) {
        const int i = list[(long long)k * n + j];
        const double* rc = pa.rec + (long long)i * kRec;
        const double xi[3] = {rc[P_X], rc[P_X + 1], rc[P_X + 2]};
        const double Hi = rc[P_H];
        double d[3];
        disp(ph, xi, xj[0], xj[1], xj[2], d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(r < Hi)) continue;   // j is not in i's gather set
        double LE[9], lS[15], dphi[5];
        for (int q = 0; q < 9; q++) LE[q] = rc[P_LE + q];
        for (int q = 0; q < 15; q++) lS[q] = rc[P_LS + q];
        for (int f = 0; f < 5; f++) dphi[f] = phi_j[f] - rc[P_PHI + f];
        double t[5], ld[3], lpsi, W, dWH;
        grad_pair_terms(d, r, Hi, rc[P_V], LE, lS, dphi, t, ld, lpsi, W, dWH);
        for (int f = 0; f < 5; f++) lphi[f] += t[f];
        for (int c = 0; c < 3; c++) lx[c] += ld[c];
        // i's limiter terms addressed to j: its length (j the farthest) and extrema
        const int4* ixp = (const int4*)(pa.lix + (long long)i * 16);
        const int4 q0 = ixp[0], q1 = ixp[1], q2 = ixp[2];
        const int ix[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
        bool any = false;
        for (int q = 0; q < 11; q++) any |= ix[q] == j;
        if (any) {
            const double* lv = pa.lval + (long long)i * 12;
            if (ix[0] == j && r > 0.0) {
                const double lhalf = lv[L_HALF];
                for (int c = 0; c < 3; c++) lx[c] += 0.5 * lhalf * d[c] / r;
            }
            for (int f = 0; f < 5; f++) {
                if (ix[1 + f] == j) lphi[f] += lv[L_MAX + f];
                if (ix[6 + f] == j) lphi[f] += lv[L_MIN + f];
            }
        }
    }
    for (int f = 0; f < 5; f++) aj.acc_phi[f * n + j] += lphi[f];
    for (int c = 0; c < 3; c++) aj.acc_x[c * n + j] += lx[c];
}

// ---------------------------------------------- kernel-length reverse and outputs
// Same split: part one (per i) finishes the outputs of i, the factor of its
// radial terms and its own side; part two (per j) adds the terms of the pairs
// whose gather set holds j.  Record: x, y, z, H, factor (in the first slots of
// the gradient record).
__global__ __launch_bounds__(256) void k_adj_length_own(PassArrays a, Phys ph, const int* __restrict__ gcount,
                                                         const int* __restrict__ list, AdjArrays aj, PullArrays pa,
                                                         double* __restrict__ out_v, double* __restrict__ out_u) {
    const int i = xcd_block_adj() * 256 + threadIdx.x;
    if (i >= a.n) return;
    const long long n = a.n;
    const double xi[3] = {a.x[i], a.y[i], a.z[i]};
    const double Hi = a.H[i], nki = a.nk[i], mi = a.m[i], ui = a.u[i];
    const double rho_i = mi * nki;
    const double lP = aj.acc_phi[4 * n + i];
    const double lrho = aj.acc_phi[0 * n + i] + (ph.gamma - 1.0) * ui * lP;
    out_u[i] = (ph.gamma - 1.0) * rho_i * lP;
    for (int c = 0; c < 3; c++) out_v[c * n + i] = aj.acc_phi[(1 + c) * n + i];
    const double ln = mi * lrho - aj.acc_V[i] / (nki * nki);
    const int cnum = gcount[i];
    // sums over the gather set (self term: r = 0, w(0) = 1, q w'(q) = 0)
    double sqdw = 0.0;
    int jn = cnum > 0 ? list[i] : 0;   // the next list entry, loaded one neighbour ahead
    for (int k = 0; k < cnum; k++) {
        const int j = jn;
        if (k + 1 < cnum) jn = list[(long long)(k + 1) * n + i];
        double d[3];
        disp(ph, xi, a.x[j], a.y[j], a.z[j], d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        sqdw += spline_qdw(r / Hi);
    }
    const double nrm = kernel_norm(Hi);
    // dn/dH = sum_j dW/dH = -(3 n + nrm sum q w') / H
    const double dndH = -(3.0 * nki + nrm * sqdw) / Hi;
    const double lH = aj.acc_H[i] + ln * dndH;
    // Phi(H) = (32/3) sum w(r/H) - N, dPhi/dH = -(32/3) sum q w' / H
    const double c32 = 32.0 / 3.0;
    const double PhiH = -c32 * sqdw / Hi;
    const double kift = -lH / PhiH;   // dH = -dPhi / PhiH
    // dn/dr = nrm w' / H ; dPhi/dr = (32/3) w' / H
    const double fac = (ln * nrm + kift * c32) / Hi;
    double* rc = pa.rec + (long long)i * kRec;
    rc[P_X] = xi[0];
    rc[P_X + 1] = xi[1];
    rc[P_X + 2] = xi[2];
    rc[P_H] = Hi;
    rc[P_V] = fac;
    double lxi[3] = {0.0, 0.0, 0.0};
    jn = cnum > 0 ? list[i] : 0;   // the next list entry, loaded one neighbour ahead
    for (int k = 0; k < cnum; k++) {
        const int j = jn;
        if (k + 1 < cnum) jn = list[(long long)(k + 1) * n + i];
        double d[3];
        disp(ph, xi, a.x[j], a.y[j], a.z[j], d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(r > 0.0)) continue;
        const double q = r / Hi;
        const double lr = fac * (spline_qdw(q) / q);   // w'(q)
        for (int c = 0; c < 3; c++) lxi[c] -= lr * d[c] / r;
    }
    for (int c = 0; c < 3; c++) pa.own[(5 + c) * n + i] = lxi[c];
}

__global__ __launch_bounds__(256) void k_adj_length_pull(PassArrays a, Phys ph, const int* __restrict__ counts,
                                                          const int* __restrict__ list, AdjArrays aj, PullArrays pa) {
    const int j = xcd_block_adj() * 256 + threadIdx.x;
    if (j >= a.n) return;
    const long long n = a.n;
    const double xj[3] = {a.x[j], a.y[j], a.z[j]};
    double lx[3];
    for (int c = 0; c < 3; c++) lx[c] = pa.own[(5 + c) * n + j];
    const int cnum = counts[j];
    for (int k = 0; k < cnum; k++) {
        const int i = list[(long long)k * n + j];
        const double* rc = pa.rec + (long long)i * kRec;
        const double xi[3] = {rc[P_X], rc[P_X + 1], rc[P_X + 2]};
        const double Hi = rc[P_H];
        double d[3];
        disp(ph, xi, xj[0], xj[1], xj[2], d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(r < Hi) || !(r > 0.0)) continue;
        const double q = r / Hi;
        const double lr = rc[P_V] * (spline_qdw(q) / q);
        for (int c = 0; c < 3; c++) lx[c] += lr * d[c] / r;
    }
    for (int c = 0; c < 3; c++) aj.acc_x[c * n + j] += lx[c];
}

void launch_pass_adjoint(const PassArrays& a, const Phys& ph, const int* counts, const int* gcount,
                         const int* list, const double* lam_dp, const double* lam_dE, double* scratch,
                         double* out_x, double* out_v, double* out_u, hipStream_t s) {
    const long long n = a.n;
    AdjArrays aj;
    aj.acc_x = out_x;
    aj.acc_phi = scratch;
    aj.acc_H = scratch + 5 * n;
    aj.acc_V = scratch + 6 * n;
    aj.acc_B = scratch + 7 * n;
    aj.acc_g = scratch + 13 * n;
    PullArrays pa;
    pa.rec = scratch + kAdjPullOffset * n;
    pa.own = pa.rec + kAdjRec * n;
    pa.lix = (int*)(pa.own + kAdjOwn * n);   // 16 int32 = 8 doubles per particle
    pa.lval = pa.own + (kAdjOwn + 8) * n;
    const int blocks = (int)((n + 255) / 256);
    k_adj_side_pack<<<blocks, 256, 0, s>>>(a, lam_dp, lam_dE, pa.rec);
    k_adj_pairs<<<blocks, 256, 0, s>>>(a, ph, counts, list, pa.rec, aj);
    k_adj_grad_own<<<blocks, 256, 0, s>>>(a, ph, gcount, list, aj, pa);
    k_adj_grad_pull<<<blocks, 256, 0, s>>>(a, ph, counts, list, aj, pa);
    k_adj_length_own<<<blocks, 256, 0, s>>>(a, ph, gcount, list, aj, pa, out_v, out_u);
    k_adj_length_pull<<<blocks, 256, 0, s>>>(a, ph, counts, list, aj, pa);
}

// ------------------------------------------------------------ step reverse
// Forward step (h = dt/2), per particle:
//   E0 = m (u + |v|^2/2); v1 = v + h p/m; E1 = E0 + h e; x' = wrap(x + dt v1)
//   vp = v1 + h p/m; Ep = E1 + h e; up = max(Ep/m - |vp|^2/2, floor)
//   (p', e') = pass(x', vp, up)
//   v' = v1 + h p'/m; E' = E1 + h e'; u' = max(E'/m - |v'|^2/2, floor)
// with p = dp/dt, e = dE/dt of the state.  Everything below is in the order
// of the recomputed step (after its re-sort).

// part 1: from the adjoints of (x', v', u', p', e') to the pass-output adjoints
// lam_p2 = lp' + h/m lv'_tot, lam_e2 = le' + h lE', plus lv1 and lE1 so far
__global__ void k_step_rev1(int n_, const double* __restrict__ m, const double* __restrict__ v1x,
                            const double* __restrict__ v1y, const double* __restrict__ v1z,
                            const double* __restrict__ Ehalf, const double* __restrict__ dp2,
                            const double* __restrict__ dE2, double dt, double u_floor, const double* __restrict__ lx,
                            const double* __restrict__ lv, const double* __restrict__ lu,
                            const double* __restrict__ lp, const double* __restrict__ le,
                            double* __restrict__ lam_p2, double* __restrict__ lam_e2, double* __restrict__ lv1,
                            double* __restrict__ lE1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_) return;
    const long long n = n_;
    const double h = 0.5 * dt, mi = m[i];
    const double v1[3] = {v1x[i], v1y[i], v1z[i]};
    double v2[3];
    for (int c = 0; c < 3; c++) v2[c] = v1[c] + h * dp2[c * n + i] / mi;
    const double E2 = Ehalf[i] + h * dE2[i];
    const double u2 = E2 / mi - 0.5 * (v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2]);
    const bool floored = u2 < u_floor;
    const double lu2 = floored ? 0.0 : lu[i];
    const double lE2 = lu2 / mi;
    for (int c = 0; c < 3; c++) {
        const double lvt = lv[c * n + i] - lu2 * v2[c];
        lam_p2[c * n + i] = lp[c * n + i] + h / mi * lvt;
        lv1[c * n + i] = lvt + dt * lx[c * n + i];   // v1 feeds v' and x'
    }
    lam_e2[i] = le[i] + h * lE2;
    lE1[i] = lE2;
}

// part 2 (recomputed order): after the pass adjoint gave (lxF, lvp, lup),
// the adjoints of the step's start state, except the term of E0 = m (u + |v|^2/2)
// in v, which needs v at the start and is added after un-permuting (part 3)
__global__ void k_step_rev2(int n_, const double* __restrict__ m, const double* __restrict__ vp,
                            const double* __restrict__ up, double dt, double u_floor,
                            const double* __restrict__ lx2, const double* __restrict__ lxF,
                            const double* __restrict__ lvp, const double* __restrict__ lup,
                            const double* __restrict__ lv1_in, const double* __restrict__ lE1_in,
                            double* __restrict__ out_lx, double* __restrict__ out_lv, double* __restrict__ out_lu,
                            double* __restrict__ out_lp, double* __restrict__ out_le, double* __restrict__ out_lE0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_) return;
    const long long n = n_;
    const double h = 0.5 * dt, mi = m[i];
    double q[3];
    for (int c = 0; c < 3; c++) q[c] = vp[c * n + i];
    const bool floored = !(up[i] > u_floor);
    const double lu_p = floored ? 0.0 : lup[i];
    const double lEp = lu_p / mi;
    const double lE1 = lE1_in[i] + lEp;     // Ep = E1 + h e
    double le0 = h * lEp + h * lE1;         // E1 = E0 + h e
    for (int c = 0; c < 3; c++) {
        const double lvpt = lvp[c * n + i] - lu_p * q[c];
        const double lv1 = lv1_in[c * n + i] + lvpt + dt * lxF[c * n + i];
        out_lx[c * n + i] = lx2[c * n + i] + lxF[c * n + i];
        out_lp[c * n + i] = h / mi * lvpt + h / mi * lv1;   // vp and v1 both take h p/m
        out_lv[c * n + i] = lv1;                            // v1 = v + h p/m
    }
    out_lu[i] = mi * lE1;
    out_le[i] = le0;
    out_lE0[i] = lE1;
}

// part 3 (start order): lv += m v lE0
__global__ void k_step_rev3(int n_, const double* __restrict__ m, const double* __restrict__ vx,
                            const double* __restrict__ vy, const double* __restrict__ vz,
                            const double* __restrict__ lE0, double* __restrict__ lv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_) return;
    const long long n = n_;
    const double t = m[i] * lE0[i];
    lv[i] += t * vx[i];
    lv[n + i] += t * vy[i];
    lv[2 * n + i] += t * vz[i];
}

// out[idx[k]] = in[k] for `count` arrays of length n (back to the pre-sort order)
__global__ void k_unpermute(int n, GatherBatch gb, const int* __restrict__ idx) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int d = idx[k];
    if (d < 0 || d >= n) return;
    for (int a = 0; a < gb.count; a++) gb.dst[a][d] = gb.src[a][k];
}

void launch_step_rev1(int n, const double* m, const double* v1x, const double* v1y, const double* v1z,
                      const double* Ehalf, const double* dp2, const double* dE2, double dt, double u_floor,
                      const double* lx, const double* lv, const double* lu, const double* lp, const double* le,
                      double* lam_p2, double* lam_e2, double* lv1, double* lE1, hipStream_t s) {
    k_step_rev1<<<(n + 255) / 256, 256, 0, s>>>(n, m, v1x, v1y, v1z, Ehalf, dp2, dE2, dt, u_floor, lx, lv, lu, lp,
                                                le, lam_p2, lam_e2, lv1, lE1);
}

void launch_step_rev2(int n, const double* m, const double* vp, const double* up, double dt, double u_floor,
                      const double* lx2, const double* lxF, const double* lvp, const double* lup, const double* lv1,
                      const double* lE1, double* out_lx, double* out_lv, double* out_lu, double* out_lp,
                      double* out_le, double* out_lE0, hipStream_t s) {
    k_step_rev2<<<(n + 255) / 256, 256, 0, s>>>(n, m, vp, up, dt, u_floor, lx2, lxF, lvp, lup, lv1, lE1, out_lx,
                                                out_lv, out_lu, out_lp, out_le, out_lE0);
}

void launch_step_rev3(int n, const double* m, const double* vx, const double* vy, const double* vz,
                      const double* lE0, double* lv, hipStream_t s) {
    k_step_rev3<<<(n + 255) / 256, 256, 0, s>>>(n, m, vx, vy, vz, lE0, lv);
}

// the used entries of each particle's flux list (k < counts[i]), for a step's tape
__global__ void k_copy_lists(int n, const int* __restrict__ counts, const int* __restrict__ src,
                             int* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = counts[i];
    for (int k = 0; k < c; k++) dst[(long long)k * n + i] = src[(long long)k * n + i];
}

void launch_copy_lists(int n, const int* counts, const int* src, int* dst, hipStream_t s) {
    k_copy_lists<<<(n + 255) / 256, 256, 0, s>>>(n, counts, src, dst);
}

void launch_unpermute(int n, const GatherBatch& gb, const int* idx, hipStream_t s) {
    k_unpermute<<<(n + 255) / 256, 256, 0, s>>>(n, gb, idx);
}

}  // namespace mfm
