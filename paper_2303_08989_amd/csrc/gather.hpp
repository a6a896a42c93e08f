// A GEMM operand read through a permutation of its tensor's index bits, so
// that the transpose of TTGT contraction and the split of Eq. 2 are one
// pass over the operand (the permuted copy is never written).
#pragma once
#include "common.hpp"

namespace qce {

// Operand P (rows x k, rows = 2^nr, k = 2^nk) of a tensor x of 2^(nr+nk)
// elements whose index bits are those of (r, l) in another order:
//   P[r][l] = x[sum_i bit_i(r) 2^rsh[i] + sum_j bit_j(l) 2^ksh[j]].
// The split stages blocks of 64 rows x 64 k-values; the tile's own index
// bits (the low min(6, nr) bits of r and min(6, nk) of l) are listed in
// tsh / tpos by increasing stride in x, so that consecutive threads load
// consecutive addresses wherever x's lowest bits fall inside the tile.
struct GatherMap {
    int nr = 0, nk = 0, nt = 0;
    int8_t rsh[32] = {}, ksh[32] = {};
    int8_t tsh[12] = {};   // stride exponent in x of tile bit b
    int8_t tpos[12] = {};  // 0..5: bit tpos of r; 6..11: bit tpos - 6 of l
};

// Checks that a map is a permutation of nr + nk bits with a consistent tile
// list (the kernel's loads stay inside x exactly when this holds).
bool gather_map_valid(const GatherMap &gm);

// The split of launch_split_panels for an operand given by a GatherMap
// (one GEMM, no batch): same panel format, mode and shift handling.
hipError_t launch_split_gather(const float2 *x, const GatherMap &gm, void *panels, const DevState *st,
                               int which, int forced_mode, int shift, hipStream_t s);

// Full contraction c[0] = sum_i x[perm(i)] * y[i] where d describes the
// permutation taking x to y's index order (as for launch_permute): x is
// read through the permutation's bit tile, y in order, products summed in
// FP32 per block into `partial`, then in a fixed order into c[0].
// permuted_dot_partials: partials needed (0: not a tiled power-of-two
// permutation, use the permute instead).
int64_t permuted_dot_partials(const PermDesc &d);
hipError_t launch_permuted_dot(const float2 *x, const float2 *y, const PermDesc &d, float2 *partial,
                               float2 *c, hipStream_t s);

}  // namespace qce
