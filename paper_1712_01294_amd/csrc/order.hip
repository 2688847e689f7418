// Particle-order utilities: whether the carried ids form a permutation, and
// their narrowing to the 32-bit indices of the scatter kernel.
#include "order.h"

namespace mfm {

__global__ void k_clear_marks(int n, int* __restrict__ marks) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) marks[i] = 0;
}

// one count per id; an id out of range sets the flag instead
__global__ void k_mark_ids(int n, const long long* __restrict__ id, int* __restrict__ marks,
                           unsigned long long* __restrict__ bad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const long long d = id[k];
    if (d < 0 || d >= n) {
        atomicOr(bad, 1ull);
        return;
    }
    atomicAdd(&marks[d], 1);
}

// every value taken exactly once (n ids in range: no value twice iff none missing)
__global__ void k_check_marks(int n, const int* __restrict__ marks, unsigned long long* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && marks[i] != 1) atomicOr(bad, 1ull);
}

__global__ void k_narrow_ids(int n, const long long* __restrict__ id, int* __restrict__ idx) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) idx[k] = (int)id[k];
}

void launch_check_perm(int n, const long long* id, int* marks, unsigned long long* bad, hipStream_t s) {
    const int blocks = (n + 255) / 256;
    k_clear_marks<<<blocks, 256, 0, s>>>(n, marks);
    k_mark_ids<<<blocks, 256, 0, s>>>(n, id, marks, bad);
    k_check_marks<<<blocks, 256, 0, s>>>(n, marks, bad);
}

void launch_narrow_ids(int n, const long long* id, int* idx, hipStream_t s) {
    k_narrow_ids<<<(n + 255) / 256, 256, 0, s>>>(n, id, idx);
}

}  // namespace mfm
