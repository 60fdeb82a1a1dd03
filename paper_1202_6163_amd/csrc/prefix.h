// Tile layout and workspace of the prefix-sum resamplers (stratified,
// systematic, multinomial) and the log-sum-exp reduction.
//
// The particles are cut into tiles of kTile consecutive weights. A first
// kernel reduces every tile to (max, sum of exp(lw - max)); the block that
// finishes last combines the partials into the tile boundaries
// B_t = C_{(t+1) kTile - 1} of the cumulative weight and the launch table of
// the second kernel. The second kernel recomputes each tile's scan on chip and
// writes ancestors (stratified/systematic: a merge of sorted draw points with
// sorted cumulative weights) or the cumulative weights (multinomial, searched
// by a third kernel).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rs {

constexpr int kTile = 1024;          // weights per tile
constexpr int kTileThreads = 256;    // threads per tile block (4 weights each)
constexpr int kChunk = 2048;         // outputs per fill block (8 per thread)
constexpr int kChunkSlack = 16;      // extra outputs a tile may own beyond its weight share

// Kinds of prefix-sum pass.
constexpr int kStratified = 0;
constexpr int kSystematic = 1;
constexpr int kMultinomial = 2;
constexpr int kLogSumExp = 4;

struct alignas(64) WsHeader {
    unsigned int counter;  // tiles finished (last block resets it to 0)
    int flags;             // OR of data flags; nonzero = table invalid
    int n_overflow;        // extra fill chunks of heavy tiles
    int acc_flags;         // flags OR-ed by the tile blocks (last block resets)
    float m;               // max lw
    float pad1;
    double W;              // total weight sum exp(lw - m)
    double delta;          // W / P
    double lse;            // m + log W
};

struct WsLayout {
    size_t header, tile_max, tile_sum, bound, overflow, cumw, total;
};

__host__ __device__ inline size_t ws_align(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline int64_t num_tiles(int64_t P) { return (P + kTile - 1) / kTile; }

__host__ __device__ inline WsLayout ws_layout(int64_t P, bool with_cumw)
{
    const int64_t n = num_tiles(P);
    WsLayout L;
    L.header = 0;
    L.tile_max = ws_align(sizeof(WsHeader));
    L.tile_sum = L.tile_max + ws_align((size_t)n * sizeof(float));
    L.bound = L.tile_sum + ws_align((size_t)n * sizeof(double));
    L.overflow = L.bound + ws_align((size_t)n * sizeof(double));
    L.cumw = L.overflow + ws_align((size_t)(n + 1) * sizeof(int32_t));
    L.total = L.cumw + (with_cumw ? ws_align((size_t)P * sizeof(double)) : 0);
    return L;
}

// Upper bound on the fill blocks beyond one per tile, used as launch size.
__host__ __device__ inline int64_t max_overflow_chunks(int64_t P)
{
    const int64_t n = num_tiles(P);
    return (P + (int64_t)(kChunkSlack + 1) * n + kChunk - 1) / kChunk + 1;
}

}  // namespace rs
