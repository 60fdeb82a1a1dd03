// Tile layout and workspace of the prefix-sum resamplers (stratified,
// systematic, multinomial) and the log-sum-exp reduction.
//
// The particles are cut into tiles of kTile consecutive weights. Launch 1
// reduces every tile to (max, sum of exp(lw - max), data flags). Launch 2 (one
// block) combines the partials into the tile boundaries B_t (the cumulative
// weight at each tile end), the number of draw points below each boundary and
// the owner tile of every kChunk-wide window of draws. Launch 3 recomputes
// each tile's scan on chip and writes ancestors and offspring
// (stratified/systematic: a merge of sorted draw points with sorted
// cumulative weights) or the cumulative weights (multinomial, searched by a
// fourth launch). Kernel boundaries order the phases, so no block waits on
// another and the workspace needs no initialisation.
//
// Up to kOnePassMaxTiles tiles the stratified/systematic resampler can also
// run as one launch (onepass_kernel in prefix.hip): every block publishes its
// tiles' (max, sum, flags) as tagged 64-bit words in the `pub` section and
// reads all of them back. The launcher clears those words with a fill kernel
// just before, and a published word is never zero, so words left by earlier
// calls (of any kind or size) are never taken for current ones and this path,
// too, needs no initialisation.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rs {

constexpr int kTile = 1024;          // weights per tile
constexpr int kTileThreads = 256;    // threads per tile block (4 weights each)
constexpr int kChunk = 2048;         // output slots per fill block (8 per thread)
constexpr int kWindow = kChunk - 4;  // draws per overflow window (see fill_body)

// Kinds of prefix-sum pass.
constexpr int kStratified = 0;
constexpr int kSystematic = 1;
constexpr int kMultinomial = 2;
constexpr int kLogSumExp = 4;
constexpr int kAdaptiveB = 5;  // log-sum-exp plus the eq. (5) iteration count

struct alignas(64) WsHeader {
    int flags;       // OR of data flags; nonzero = table invalid
    float m;         // max lw
    double W;        // total weight sum exp(lw - m)
    double delta;    // W / P
    double lse;      // m + log W
    uint32_t B;      // adaptive Metropolis iterations (eq. (5) at w_max = 1 / W)
    uint32_t pad2;
};

struct WsLayout {
    size_t header, tile_max, tile_sum, tile_flags, bound, count, win, pub, sub, guide, part,
        cumw, total;
};

__host__ __device__ inline size_t ws_align(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline int64_t num_tiles(int64_t P) { return (P + kTile - 1) / kTile; }

// kWindow-wide windows of draw indices (the unit of the fill's overflow blocks).
__host__ __device__ inline int64_t num_windows(int64_t P) { return (P + kWindow - 1) / kWindow; }

// Multinomial search: the particles are cut into kParts contiguous parts
// (one per XCD of the MI355X: each part's cumulative weights stay in that
// XCD's L2). Within part x the last C' of every group of sub_stride(P)
// particles goes to a compact array, at most kSubMax doubles per part (staged
// in LDS by the search); the groups are 16 particles (one 128-byte line) up to
// 2^20 particles and double beyond.
constexpr int kParts = 8;
constexpr int64_t kSubMax = 8192;
// Parts are whole tiles, so a part's lower bound in C' is a tile boundary.
__host__ __device__ inline int64_t part_size(int64_t P)
{
    const int64_t p = (P + kParts - 1) / kParts;
    return (p + kTile - 1) / kTile * kTile;
}
__host__ __device__ inline int64_t sub_stride(int64_t P)
{
    int64_t s = 16;
    while ((part_size(P) + s - 1) / s > kSubMax) s <<= 1;
    return s;
}
__host__ __device__ inline int64_t sub_per_part(int64_t P)
{
    const int64_t s = sub_stride(P);
    return (part_size(P) + s - 1) / s;
}
__host__ __device__ inline int64_t num_sub(int64_t P) { return kParts * sub_per_part(P); }
// The search's guide table per part: entries 0 .. sub_per_part(P) (uint16),
// padded to whole 16-byte vectors.
__host__ __device__ inline int64_t guide_stride(int64_t P) { return (sub_per_part(P) + 8) / 8 * 8; }

__host__ __device__ inline WsLayout ws_layout(int64_t P, bool with_cumw)
{
    const size_t n = (size_t)num_tiles(P);
    WsLayout L;
    L.header = 0;
    L.tile_max = ws_align(sizeof(WsHeader));
    L.tile_sum = L.tile_max + ws_align(n * sizeof(float));
    L.tile_flags = L.tile_sum + ws_align(n * sizeof(double));
    L.bound = L.tile_flags + ws_align(n * sizeof(int32_t));
    L.count = L.bound + ws_align(n * sizeof(double));
    L.win = L.count + ws_align(n * sizeof(int32_t));
    // one-pass path: three tagged words per tile
    L.pub = L.win + ws_align((size_t)num_windows(P) * sizeof(int32_t));
    // the multinomial sections (group ends, guide, draw parts, C) sit past the shared
    // ones at the same offsets whatever the kind; only the size differs
    L.sub = L.pub + ws_align(n * 3 * sizeof(uint64_t));
    L.guide = L.sub + ws_align((size_t)num_sub(P) * sizeof(double));
    L.part = L.guide + ws_align((size_t)(kParts * guide_stride(P)) * sizeof(uint16_t));
    L.cumw = L.part + ws_align((size_t)P + 16);
    L.total = with_cumw ? L.cumw + ws_align((size_t)P * sizeof(double)) : L.sub;
    return L;
}

// Fill blocks of a stratified/systematic resampling: one per tile, plus one
// per kWindow-wide window of draw indices for the draws of heavy tiles that
// do not fit in their tile block (see fill_body).
__host__ __device__ inline int64_t num_fill_blocks(int64_t P)
{
    return num_tiles(P) + num_windows(P);
}

// Up to this many tiles a fill block rebuilds all tile boundaries itself (in
// LDS) instead of reading them from a separate table launch: for small
// instances the extra launch costs more than the redundant scan, for large
// ones (measured at 1024 tiles) the other way round.
constexpr int64_t kFusedTableTiles = 64;

// The one-pass stratified/systematic launch: at most this many tiles (P <=
// 2^20), kOnePassTiles tiles per block.
constexpr int64_t kOnePassMaxTiles = 1024;
constexpr int kOnePassTiles = 2;

}  // namespace rs
