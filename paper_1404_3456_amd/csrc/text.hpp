// text.hpp -- random-access 32-position windows of the packed text (device side).
//
// Record b of the block layout holds the 2-bit codes of positions 32b .. 32b+31 (two words,
// position 32b in the top bits of the first) and their separator bits (position 32b in bit
// 31), padded to 16 bytes; launch_blocks builds it from the packed words and separator mask.
// A window starting anywhere is then two aligned 16-byte loads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace saasm {

struct Window {
    uint64_t code;  // 32 bases from position a, base a in bits 63..62
    uint32_t sep;   // separator bits of positions a .. a+31, position a in bit 31
};

// Needs records a/32 and a/32 + 1.
__device__ __forceinline__ Window window_at(const uint4 *__restrict__ blk, uint32_t a) {
    const uint32_t b = a >> 5, o = a & 31;
    const uint4 x = blk[b], y = blk[b + 1];
    const uint64_t c0 = (uint64_t(x.x) << 32) | x.y, c1 = (uint64_t(y.x) << 32) | y.y;
    Window w;
    w.code = o ? (c0 << (2 * o)) | (c1 >> (64 - 2 * o)) : c0;
    w.sep = o ? (x.z << o) | (y.z >> (32 - o)) : x.z;
    return w;
}

// 32 bases of a packed code array (16 per word, base 0 in the top bits) from base a; reads
// words a/16 .. a/16 + 2.
__device__ __forceinline__ uint64_t codes_at(const uint32_t *__restrict__ packed, uint64_t a) {
    const uint64_t w = a >> 4;
    const uint32_t o = uint32_t(a & 15);
    uint64_t x = (uint64_t(packed[w]) << 32) | packed[w + 1];
    x <<= 2 * o;
    if (o) x |= uint64_t(packed[w + 2]) >> (32 - 2 * o);
    return x;
}

}  // namespace saasm
