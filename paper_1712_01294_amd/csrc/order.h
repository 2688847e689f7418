// Launchers of the particle-order utilities: restoring the order in which the
// caller gave the particles, from the ids every reordering carries along.
#pragma once

#include <hip/hip_runtime.h>

namespace mfm {

// bad |= 1 unless id[0 .. n) holds every value 0 .. n-1 exactly once; marks
// (n ints) is scratch, cleared here
void launch_check_perm(int n, const long long* id, int* marks, unsigned long long* bad, hipStream_t s);
// idx[k] = id[k], for ids already checked to lie in 0 .. n-1
void launch_narrow_ids(int n, const long long* id, int* idx, hipStream_t s);

}  // namespace mfm
