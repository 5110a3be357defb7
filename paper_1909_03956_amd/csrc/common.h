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
//   root : a = A_1 * lambda_1 of the level-1 node that follows; meta = 0
//   node : a, b, c = h^0, h^1, h^2 with h^m = s^m_{c0} gamma^m_j (sqrt(A_j)/4) 4^-(J-j-1),
//          c0 the node's first child, s the Eq. 10 signs (a thresholded tree:
//          0 for a coefficient that is not kept)
//   leaf : a, b, c = l, m, n - 1 of the pixel centre
// meta of nodes and leaves:
//   bits 0-3   child mask (bit c set if child 4k + c exists; 0 for a leaf)
//   bits 8-12  level j
//   bits 32-63 for a node with exactly one child: the number of consecutive
//              one-child nodes that start here (this one, its child, ...);
//              they are contiguous in the stream.  0 otherwise.
struct alignas(32) TRec {
    double a, b, c;
    unsigned long long meta;
};

constexpr unsigned meta_mask(unsigned long long meta) { return (unsigned)(meta & 0xFu); }
constexpr int meta_level(unsigned long long meta) { return (int)((meta >> 8) & 31u); }
constexpr int meta_chain(unsigned long long meta) { return (int)(meta >> 32); }
constexpr unsigned long long make_meta(unsigned mask, int level, int chain) {
    return (unsigned long long)(mask & 0xFu) | ((unsigned long long)level << 8) |
           ((unsigned long long)(unsigned)chain << 32);
}

// Deferred-error bits the kernels raise in the context's status word.
enum : int { kStatusDomain = 1, kStatusNonFinite = 2 };

// Sets the thread-local message and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

}  // namespace swv
