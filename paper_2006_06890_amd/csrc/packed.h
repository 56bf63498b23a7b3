// Device side of the packed list format (EMOGI_F_PACK; the compression with
// decoding on idle GPU cores that EMOGI proposes in Sec. 6).  A list is cut
// into blocks of 64 ids; a block is its first id as a whole 32-bit word, the
// gaps to its other ids at the list's gap width w, then (with weights) its
// weights at the list's weight width ww, each part bit-packed into whole
// words.  Every block but a list's last is full, so block k of a list
// starting at word off starts at word off + k * packed_block_words(w, ww).
#pragma once

#include "internal.h"
#include "wave.h"

#include <type_traits>

namespace emogi {

// Tag for packed lists in the ColT slot of the kernels that read lists.
struct PackedCol {
    uint32_t x;
};
template <class ColT>
constexpr bool kPacked = std::is_same<ColT, PackedCol>::value;

// Words of a full packed block: first id, 63 gaps of w bits, 64 weights of ww bits.
__device__ __forceinline__ uint32_t packed_block_words(uint32_t w, uint32_t ww) {
    return 1u + (63u * w + 31u) / 32u + 2u * ww;
}

// Id words of a block of cnt (1..64) ids at gap width w (at most 64 for w <= 32).
__device__ __forceinline__ uint32_t packed_id_words(uint32_t cnt, uint32_t w) {
    return 1u + ((cnt - 1u) * w + 31u) / 32u;
}

// Weight words of a block of cnt (1..64) weights at width ww (at most 64).
__device__ __forceinline__ uint32_t packed_block_weight_words(uint32_t cnt, uint32_t ww) {
    return (cnt * ww + 31u) / 32u;
}

// Weight words of a packed list of d ids at weight width ww.
__device__ __forceinline__ uint64_t packed_weight_words(uint64_t d, uint32_t ww) {
    if (d == 0) return 0;
    const uint64_t nb = (d + 63) / 64, last = d - (nb - 1) * 64;
    return (nb - 1) * 2 * uint64_t(ww) + (last * ww + 31) / 32;
}

// Inclusive prefix sum over the 64 lanes (every lane calls it), on DPP lane
// moves inside the VALU adds (no LDS traffic): shifts by 1, 2, 4 and 8 lanes
// within each row of 16 (lanes shifted in from outside the row read 0) give
// each row's own prefix; then lane 15's sum is broadcast into rows 1 and 3
// and lane 31's (the sum of rows 0-1) into rows 2 and 3.  Masked-off rows
// take the `old` value 0.
__device__ __forceinline__ uint32_t wave_prefix_sum(uint32_t x) {
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 1, 0xf, 0xf, true));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 2, 0xf, 0xf, true));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 4, 0xf, 0xf, true));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 8, 0xf, 0xf, true));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowBcast15, 0xa, 0xf, false));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowBcast31, 0xc, 0xf, false));
    return x;
}

// Lane `src` (taken modulo 64) of x, through the LDS crossbar (no memory
// access).  Every lane must be active.
__device__ __forceinline__ uint32_t lane_word(uint32_t x, uint32_t src) {
    return uint32_t(__builtin_amdgcn_ds_bpermute(int(src << 2), int(x)));
}

// The `w`-bit field at bit `sh` of the 64-bit window hi:lo.
__device__ __forceinline__ uint32_t packed_field(uint32_t lo, uint32_t hi, uint32_t sh, uint32_t w) {
    const uint64_t word = (uint64_t(hi) << 32) | lo;
    return uint32_t((word >> sh) & ((uint64_t(1) << w) - 1));
}

// The f-th w-bit field of a bit string whose 32-bit word j sits in lane
// `first + j` (word f * w / 32 and the next one are gathered from their lanes).
__device__ __forceinline__ uint32_t lane_field(uint32_t word, uint32_t first, uint32_t f, uint32_t w) {
    const uint32_t o = f * w, j = first + (o >> 5);
    return packed_field(lane_word(word, j), lane_word(word, j + 1), o & 31u, w);
}

// Decodes a block's ids from its id words, loaded one per lane (lane j holds
// word j, j < packed_id_words(cnt, w); 0 above): lane l < cnt returns the
// block's l-th id (lanes at or above cnt return values to be ignored).
// Every lane calls it.
__device__ __forceinline__ uint32_t packed_ids(uint32_t word, uint32_t w, uint32_t cnt, int lane) {
    const uint32_t gap = lane_field(word, 1u, uint32_t(lane) - 1u, w);  // lane 0's is discarded
    const uint32_t x = lane == 0 ? word : (uint32_t(lane) < cnt ? gap : 0u);
    return wave_prefix_sum(x);  // first id + the gaps up to each lane
}

// Decodes a block's weights from its weight words, loaded one per lane
// likewise: lane l returns weight l.  Every lane calls it.
__device__ __forceinline__ uint32_t packed_weights(uint32_t word, uint32_t ww, int lane) {
    return lane_field(word, 0u, uint32_t(lane), ww);
}

// Loads and decodes block `wb` (its first word) of a list holding `cnt` ids
// in it (1..64): lane l < cnt returns the block's l-th id and, when `ww` is
// not 0 and `wt` is set, its weight.  Each word is loaded once, by one lane.
// Every lane of the wave calls it.
__device__ __forceinline__ uint32_t packed_block(const uint32_t *pk, uint64_t wb, uint32_t w, uint32_t ww,
                                                 uint32_t cnt, int lane, uint32_t *wt) {
    const uint32_t l = uint32_t(lane), idw = packed_id_words(cnt, w);
    const uint32_t idword = l < idw ? pk[wb + l] : 0u;
    if (wt) {
        const uint32_t wword = l < packed_block_weight_words(cnt, ww) ? pk[wb + idw + l] : 0u;
        *wt = packed_weights(wword, ww, lane);
    }
    return packed_ids(idword, w, cnt, lane);
}

}  // namespace emogi
