// Internal definitions shared by the host runtime and the kernels of libswvis.
#pragma once

#include <cstdint>
#include <string>

#include "../../include/swvis.h"

namespace swv {

// One packed component as the direct kernels read it: 32 bytes, so a wave
// fetches a whole record with one scalar load.  nm1 = n - 1.
struct alignas(32) Comp {
    double l, m, nm1, I;
};

// One record of the depth-first tree stream (32 bytes).
//   root : a = A_1 * lambda_1 of the level-1 node that follows
//   node : a, b, c = gamma^0, gamma^1, gamma^2; meta = 4-bit child mask
//   leaf : a, b, c = l, m, n - 1 of the pixel centre
struct alignas(32) TRec {
    double a, b, c;
    unsigned long long meta;
};

// Deferred-error bits the kernels raise in the context's status word.
enum : int { kStatusDomain = 1, kStatusNonFinite = 2 };

// Sets the thread-local message and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

}  // namespace swv
