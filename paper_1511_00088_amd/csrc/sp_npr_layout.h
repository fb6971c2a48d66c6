// Placement of the NPR path matrices in LDS (sp_npr.hip): a hypercube's 256 corner-pair matrices are held as
// nine planes, one per matrix element, of NPR_PLANE 16-byte words each.
#pragma once

#include <hip/hip_runtime.h>

namespace sp {

// Plane length: 256 pairs and one word of padding, so that one pair's elements in different planes fall in
// different LDS banks.
constexpr int NPR_PLANE = 257;

// Position of the corner pair (X, Y) in a plane: X * 16 + (Y xor h(X)), with h(X) the product of X and x in
// GF(16) (modulus x^4 + x + 1). Both h and X -> X xor h(X) are one to one, so the pairs that a wavefront
// touches at once land in distinct LDS banks: (X, Y) for many X and one Y (the contraction), and (X, X xor d)
// for many X and one corner difference d (the path recursion's reads and writes).
__host__ __device__ __forceinline__ int ppos(int X, int Y) {
    const int h = ((X << 1) ^ ((X & 8) ? 0x13 : 0)) & 15;
    return X * 16 + (Y ^ h);
}

}  // namespace sp
