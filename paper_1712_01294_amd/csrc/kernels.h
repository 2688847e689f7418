// Host-side launchers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mfm {

constexpr int kGatherMax = 20;
constexpr int kRCap = 160;  // radii slots per particle in the kernel-length solve

// up to kGatherMax arrays of 8-byte elements reordered by one launch: dst[i] = src[idx[i]]
struct GatherBatch {
    int count;
    const unsigned long long* src[kGatherMax];
    unsigned long long* dst[kGatherMax];
};

// particle arrays seen by the pass kernels (sorted order)
struct PassArrays {
    int n;
    const double *x, *y, *z, *m, *vx, *vy, *vz, *u;
    double *H, *nk, *V;
    double *B, *rho, *P, *grad, *alpha;
    double *dp, *dE, *vsig;
    double *dm;   // finite-volume form only
};

// tree.hip
long long scan_tmp_ints(long long m);
void exclusive_scan(int m, const int* in, int* out, int* tmp, hipStream_t s);
void radix_sort(int n, int bits, unsigned long long* keys, int* vals, unsigned long long* ktmp,
                int* vtmp, int* hist, int* scan_tmp, hipStream_t s);
void launch_keys(int n, const double* x, const double* y, const double* z, const TreeDesc& td,
                 unsigned long long* keys, int* idx, hipStream_t s);
void launch_gather(int n, const GatherBatch& gb, const int* idx, hipStream_t s);
void launch_fill_u64(long long m, unsigned long long* p, unsigned long long v, hipStream_t s);
// all counter copies to their start values in one launch
void launch_reset_counters(Counters* c, hipStream_t s);
// dst[a][k] = src[a][k], k < n, for the arrays of the batch in one launch
void launch_copy_batch(int n, const GatherBatch& gb, hipStream_t s);
void launch_tables(int n, const unsigned long long* keys, const TreeDesc& td, int2* tab, hipStream_t s);
// clears the entries that launch_tables wrote for the same n sorted keys
void launch_untables(int n, const unsigned long long* keys, const TreeDesc& td, int2* tab, hipStream_t s);
void launch_pos4(int n, const double* x, const double* y, const double* z, double4* pos, hipStream_t s);

// pass.hip
void launch_solve_h(const PassArrays& a, const TreeDesc& td, const int2* tab,
                    const double4* pos, const Phys& ph, Counters* cnt, double* rl, int* list, int* gcount,
                    int* counts, int* fb_list, unsigned long long* fb_count, int* fb2_list,
                    unsigned long long* fb2_count, hipEvent_t t0, hipEvent_t t1, hipStream_t s);
// flux-list tail entries per particle held in its contiguous tail buffer
constexpr int kTailBuf = 32;
void launch_gradients(const PassArrays& a, const Phys& ph, const int* gcount, int* counts, int* list, int* tails,
                      int mixed, double4* prim, void* rec, Counters* cnt, hipEvent_t t0, hipEvent_t t1,
                      hipStream_t s);
void launch_fluxes(const PassArrays& a, const Phys& ph, const int* counts, const int* list,
                   int mixed, int mfv, const void* rec, Counters* cnt, hipStream_t s);
// hierarchical steps: the pairs of level >= lmin (level = the finer bin of the
// two), their per-level sums into lev[(l * 4 + c) * n + i] (FP64 records, MFM)
constexpr int kMaxBin = 7;
// (particle i's sums at column home[i] of lev; home null: column i)
void launch_fluxes_levels(const PassArrays& a, const Phys& ph, const int* counts, const int* list, const void* rec,
                          Counters* cnt, const long long* bin, int lmin, int nlev, double* lev,
                          const long long* home, hipStream_t s);

// hierarchical steps with active subsets (FP64 records, MFM): a particle's
// mode at a sub-step boundary is kModeSolve when its bin is due (new kernel
// length and gradients), kModeKept when it keeps them but an active particle
// may lie within its kernel length (it lists its gather set), kModeNone
// otherwise (no gather list; it enters only the lists of active particles
// that reach it)
constexpr unsigned char kModeNone = 0, kModeSolve = 1, kModeKept = 2;
// (the cell tables may be those of an earlier build, with particles moved by
// at most *pad since: every scan reaches that much further)
void launch_solve_h_active(const PassArrays& a, const TreeDesc& td, const int2* tab, const double4* pos,
                           const Phys& ph, Counters* cnt, const unsigned char* mode, const double* pad, double* rl,
                           int* list, int* gcount, int* counts, int* fb_list, unsigned long long* fb_count,
                           int* fb2_list, unsigned long long* fb2_count, hipStream_t s);
// (the new gradient matrices and limited gradients of the active particles, and
// the kept ones read for the records, at column home[i] of B and grad)
void launch_gradients_active(const PassArrays& a, const Phys& ph, const unsigned char* mode, const long long* home,
                             const int* gcount, int* counts, int* list, int* tails, double4* prim, void* rec,
                             Counters* cnt, hipStream_t s);
// step.hip
void launch_kick_drift(const PassArrays& a, const Phys& ph, double dt, double u_floor,
                       double* vp, double* up, double* Ehalf, hipStream_t s);
void launch_kick2(const PassArrays& a, double dt, double u_floor, const double* Ehalf,
                  double* u, Counters* cnt, hipStream_t s);
void launch_kick_drift_mfv(const PassArrays& a, const Phys& ph, double dt, double u_floor,
                           double* vp, double* up, double* Ehalf, double* mp, hipStream_t s);
void launch_kick2_mfv(const PassArrays& a, double dt, double u_floor, const double* Ehalf,
                      double* u, Counters* cnt, hipStream_t s);
void launch_dt_min(int n, const double* H, const double* vsig, double* partial, int nparts,
                   double* out, hipStream_t s);
int dt_min_parts(int n);
// hierarchical steps: E = m (u + |v|^2/2) into E and the opening kicks of every
// level (begin, rates in the particles' order); kicks of the levels >= lmin
// with their sums in lev, each of weight T / 2^(l+1), applied `times` times
// (v and E in place); drift x += dt v; predicted v, u of the pass; the
// recovery u = E/m - |v|^2/2 (floored) at the end.  Within a system step a
// particle's rates stay in the column of lev where it stood at the step's
// start, home[i], which travels with the particle (launch_iota sets it).
void launch_hier_begin(int n, const double* m, double* vx, double* vy, double* vz, const double* u, double* E,
                       const double* lev, int nlev, double T, hipStream_t s);
void launch_hier_kick(int n, const double* m, double* vx, double* vy, double* vz, double* E, const double* lev,
                      const long long* home, int lmin, int nlev, double T, int times, hipStream_t s);
// drift: with wrap the positions are wrapped into the box; with moved (n + 1
// doubles) each particle's path length since the last build accumulates in
// moved[i] and their largest in moved[n] (positive doubles ordered as integers)
void launch_hier_drift(const PassArrays& a, const Phys& ph, double dt, int wrap, double* moved, hipStream_t s);
void launch_hier_predict(int n, const double* m, const double* vx, const double* vy, const double* vz,
                         const double* E, const double* lev, const long long* home, int lmin, int nlev, double T,
                         double u_floor, double* vp, double* up, hipStream_t s);
void launch_iota(int n, long long* v, hipStream_t s);
// *bad |= 1 when some bin lies outside 0 .. max_bin
void launch_check_bins(int n, const long long* bins, int max_bin, unsigned long long* bad, hipStream_t s);
// one sweep of the neighbour time-step limiter over the flux lists:
// out[i] = max(bin[i], max over i's flux neighbours j of bin[j] - 1); *raised
// += the number of bins it raised
void launch_limit_bins(int n, int cap, const int* counts, const int* list, const long long* bin, long long* out,
                       unsigned long long* raised, hipStream_t s);
// *diff |= 2 when some particle's (x, y, z, H) differs bit for bit from
// prim[4 i] (the packed neighbour record of the last gradient pass)
void launch_same_positions(int n, const double* x, const double* y, const double* z, const double* H,
                           const double4* prim, unsigned long long* diff, hipStream_t s);
void launch_reset_counts(int n, const int* gcount, int* counts, hipStream_t s);
// the modes of one sub-step boundary: the cells (every level) of the due
// particles are marked in marks (one bit per table entry, cleared here), and
// a particle that is not due is kModeKept when the 3x3x3 cells around it, on
// the finest level whose cells are at least its H wide, hold a mark; a
// kModeNone particle's gather and list counts are set to zero
void launch_hier_modes(int n, const double* x, const double* y, const double* z, const double* H,
                       const long long* bins, int lmin, const TreeDesc& td, long long tab_len, unsigned* marks,
                       unsigned char* mode, int* gcount, int* counts, hipStream_t s);
void launch_hier_finish(int n, const double* m, const double* vx, const double* vy, const double* vz,
                        const double* E, double u_floor, double* u, Counters* cnt, hipStream_t s);

// adjoint.hip
// Adjoint scratch, doubles per particle: 0-27 pass accumulators, 28-55 step
// reverse, then the per-particle records the pass reverse pulls through the
// flux lists (kAdjRec) and its own-side terms (kAdjOwn), then the limiter
// terms part one addresses to single neighbours (kAdjLim: 16 int32 indices and
// 12 values per particle).
constexpr int kAdjRec = 36;
constexpr int kAdjOwn = 8;
constexpr int kAdjLim = 20;
constexpr int kAdjPullOffset = 56;
constexpr int kAdjSlots = kAdjPullOffset + kAdjRec + kAdjOwn + kAdjLim;

void launch_pass_adjoint(const PassArrays& a, const Phys& ph, const int* counts, const int* gcount,
                         const int* list, const double* lam_dp, const double* lam_dE, double* scratch,
                         double* out_x, double* out_v, double* out_u, hipStream_t s);
void launch_step_rev1(int n, const double* m, const double* v1x, const double* v1y, const double* v1z,
                      const double* Ehalf, const double* dp2, const double* dE2, double dt, double u_floor,
                      const double* lx, const double* lv, const double* lu, const double* lp, const double* le,
                      double* lam_p2, double* lam_e2, double* lv1, double* lE1, hipStream_t s);
void launch_step_rev2(int n, const double* m, const double* vp, const double* up, double dt, double u_floor,
                      const double* lx2, const double* lxF, const double* lvp, const double* lup, const double* lv1,
                      const double* lE1, double* out_lx, double* out_lv, double* out_lu, double* out_lp,
                      double* out_le, double* out_lE0, hipStream_t s);
void launch_step_rev3(int n, const double* m, const double* vx, const double* vy, const double* vz,
                      const double* lE0, double* lv, hipStream_t s);
void launch_unpermute(int n, const GatherBatch& gb, const int* idx, hipStream_t s);
void launch_copy_lists(int n, const int* counts, const int* src, int* dst, hipStream_t s);

}  // namespace mfm
