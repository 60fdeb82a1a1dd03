// Host side of batched resampling: validation of the instances, work-list
// construction (items sorted by decreasing cost so the round-robin deal of
// the persistent grids stays balanced) and the upload of the plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "launch.h"
#include "prefix.h"
#include "resample.h"

namespace {

constexpr int64_t kMaxP = 2147483647;

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

rs_batch_tuning tuning_or_default(const rs_batch_tuning *t)
{
    if (t) return *t;
    return rs_batch_tuning{1024, 8, 8192, 0};
}

bool valid_tuning(const rs_batch_tuning &t)
{
    const bool cpi = t.chains_per_item == 256 || t.chains_per_item == 512 ||
                     t.chains_per_item == 1024 || t.chains_per_item == 2048;
    const bool un = t.unroll == 2 || t.unroll == 4 || t.unroll == 8 || t.unroll == 16;
    return cpi && un && t.lds_max_p >= 0 && t.lds_max_p <= 32768 && t.blocks >= 0;
}

bool valid_instance(const rs_instance &d)
{
    if (d.P < 0 || d.P > kMaxP) return false;
    if (d.P == 0) return true;
    const bool metro = d.kind == RS_METROPOLIS || d.kind == RS_METROPOLIS_ADAPTIVE;
    if (!metro && d.kind != RS_STRATIFIED && d.kind != RS_SYSTEMATIC) return false;
    if (d.kind == RS_METROPOLIS_ADAPTIVE && !(d.eps > 0.0)) return false;
    // Metropolis writes ancestors; stratified/systematic ancestors and/or offspring; the
    // state copy reads the ancestors
    if (!d.lw || (metro && !d.anc) || (!d.anc && !d.off)) return false;
    if (d.off && metro) return false;
    if (d.x_in && !d.anc) return false;
    const size_t p = (size_t)d.P;
    if (d.anc && overlaps(d.lw, 4 * p, d.anc, 4 * p)) return false;
    if (d.off && (overlaps(d.lw, 4 * p, d.off, 4 * p) || (d.anc && overlaps(d.anc, 4 * p, d.off, 4 * p))))
        return false;
    if (d.x_in) {
        if (!d.x_out || d.D < 1) return false;
        const size_t rows = p * (size_t)d.D * sizeof(float);
        if (overlaps(d.x_in, rows, d.x_out, rows) || overlaps(d.anc, 4 * p, d.x_out, rows) ||
            overlaps(d.lw, 4 * p, d.x_out, rows) || (d.off && overlaps(d.off, 4 * p, d.x_out, rows)))
            return false;
    }
    return true;
}

bool is_prefix(const rs_instance &d) { return d.kind == RS_STRATIFIED || d.kind == RS_SYSTEMATIC; }

// Instances with a tile reduction and a table: the prefix resamplers, and
// adaptive Metropolis (its table leaves eq. (5)'s B in the workspace header).
bool has_table(const rs_instance &d) { return is_prefix(d) || d.kind == RS_METROPOLIS_ADAPTIVE; }

struct Layout {
    int32_t n_tile = 0, n_table = 0, n_main = 0;
    int64_t max_tiles = 0;
    size_t off_tile = 0, off_table = 0, off_main = 0, bytes = 0;
};

bool layout_of(const rs_instance *d, int32_t n, const rs_batch_tuning &t, Layout *L)
{
    int64_t tiles = 0, tables = 0, mains = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (!valid_instance(d[k])) return false;
        if (d[k].P == 0) continue;
        if (has_table(d[k])) {
            const int64_t nt = rs::num_tiles(d[k].P);
            tiles += nt;
            tables += 1;
            L->max_tiles = std::max(L->max_tiles, nt);
        }
        if (is_prefix(d[k])) {
            mains += rs::num_fill_blocks(d[k].P);
        } else {
            mains += (d[k].P + t.chains_per_item - 1) / t.chains_per_item;
        }
    }
    if (tiles > INT32_MAX || mains > INT32_MAX) return false;
    L->n_tile = (int32_t)tiles;
    L->n_table = (int32_t)tables;
    L->n_main = (int32_t)mains;
    L->off_tile = al((size_t)n * sizeof(rs::BatchInstance));
    L->off_table = L->off_tile + al((size_t)tiles * sizeof(int2));
    L->off_main = L->off_table + al((size_t)tables * sizeof(int32_t));
    L->bytes = L->off_main + al((size_t)mains * sizeof(int2));
    return true;
}

}  // namespace

extern "C" {

size_t rs_batch_plan_bytes(const rs_instance *descs, int32_t n, const rs_batch_tuning *t)
{
    const rs_batch_tuning tu = tuning_or_default(t);
    if (!descs || n < 1 || !valid_tuning(tu)) return 0;
    Layout L;
    return layout_of(descs, n, tu, &L) ? L.bytes : 0;
}

size_t rs_batch_workspace_bytes(const rs_instance *descs, int32_t n)
{
    if (!descs || n < 1) return 0;
    size_t total = 0;
    for (int32_t k = 0; k < n; ++k)
        if (descs[k].P > 0 && has_table(descs[k]))
            total += al(rs_workspace_bytes(descs[k].P, descs[k].kind));
    return total;
}

int rs_batch_plan_init(rs_batch_plan *plan, const rs_instance *descs, int32_t n,
                       const rs_batch_tuning *t, void *plan_dev, size_t plan_bytes, void *ws,
                       size_t ws_bytes, void *host_staging, hipStream_t stream)
{
    const rs_batch_tuning tu = tuning_or_default(t);
    if (!plan || !descs || n < 1 || !plan_dev || !valid_tuning(tu)) return RS_EINVAL;
    Layout L;
    if (!layout_of(descs, n, tu, &L)) return RS_EINVAL;
    if (plan_bytes < L.bytes) return RS_EWORKSPACE;
    const size_t need_ws = rs_batch_workspace_bytes(descs, n);
    if (need_ws > 0 && (!ws || ws_bytes < need_ws)) return RS_EWORKSPACE;
    if (need_ws > 0 && ((uintptr_t)ws & 255u)) return RS_EINVAL;  // 256-byte aligned sections

    std::vector<unsigned char> local;
    unsigned char *host = static_cast<unsigned char *>(host_staging);
    if (!host) {
        local.assign(L.bytes, 0);
        host = local.data();
    }
    auto *insts = reinterpret_cast<rs::BatchInstance *>(host);
    auto *tile_items = reinterpret_cast<int2 *>(host + L.off_tile);
    auto *table_items = reinterpret_cast<int32_t *>(host + L.off_table);
    auto *main_items = reinterpret_cast<int2 *>(host + L.off_main);

    struct Costed {
        int2 item;
        double cost;
    };
    std::vector<Costed> mains;
    mains.reserve((size_t)L.n_main);
    size_t ws_off = 0;
    int32_t nt = 0, nb = 0;
    for (int32_t k = 0; k < n; ++k) {
        const rs_instance &d = descs[k];
        rs::BatchInstance &I = insts[k];
        I.lw = d.lw;
        I.anc = d.anc;
        I.off = d.off;
        I.x_in = d.x_in;
        I.x_out = d.x_in ? d.x_out : nullptr;
        I.status = d.status;
        I.ws = nullptr;
        I.P = d.P;
        I.seed = d.seed;
        I.B = d.B;
        I.instance = d.instance;
        I.D = d.x_in ? d.D : 0;
        I.kind = d.kind;
        I.eps = d.kind == RS_METROPOLIS_ADAPTIVE ? d.eps : 0.0;
        if (d.P == 0) continue;
        const int64_t tiles = rs::num_tiles(d.P);
        if (has_table(d)) {
            I.ws = static_cast<char *>(ws) + ws_off;
            ws_off += al(rs_workspace_bytes(d.P, d.kind));
            for (int64_t q = 0; q < tiles; ++q) tile_items[nt++] = make_int2(k, (int)q);
            table_items[nb++] = k;
        }
        if (is_prefix(d)) {
            const int64_t fills = rs::num_fill_blocks(d.P);
            for (int64_t g = 0; g < fills; ++g)
                mains.push_back({make_int2(k, (int)g), g < tiles ? 4096.0 : 64.0});
        } else {
            const int64_t items = (d.P + tu.chains_per_item - 1) / tu.chains_per_item;
            for (int64_t q = 0; q < items; ++q) {
                const int64_t chains = std::min<int64_t>(tu.chains_per_item, d.P - q * tu.chains_per_item);
                mains.push_back({make_int2(k, (int)q), (double)chains * (double)(d.B + 4)});
            }
        }
    }
    std::stable_sort(mains.begin(), mains.end(),
                     [](const Costed &a, const Costed &b) { return a.cost > b.cost; });
    for (size_t q = 0; q < mains.size(); ++q) main_items[q] = mains[q].item;

    hipError_t e = hipMemcpyAsync(plan_dev, host, L.bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !host_staging) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        rs::record_hip_error(e);
        return RS_EHIP;
    }

    int blocks = tu.blocks;
    if (blocks == 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        blocks = 8 * std::max(cus, 1);
    }
    std::memset(plan, 0, sizeof(*plan));
    plan->dev = plan_dev;
    plan->n_instances = n;
    plan->n_tile_items = L.n_tile;
    plan->n_table_items = L.n_table;
    plan->n_main_items = L.n_main;
    plan->blocks = blocks;
    plan->unroll = tu.unroll;
    plan->chains_per_item = tu.chains_per_item;
    plan->lds_max_p = tu.lds_max_p;
    plan->max_table_tiles = L.max_tiles;
    plan->off_tile_items = L.off_tile;
    plan->off_table_items = L.off_table;
    plan->off_main_items = L.off_main;
    plan->smem_main = (uint64_t)(rs::kChunk * sizeof(int32_t) +
                                 std::max<size_t>(rs::kTile * sizeof(double),
                                                  (size_t)tu.lds_max_p * sizeof(float)));
    return RS_OK;
}

int resample_batch(const rs_batch_plan *plan, hipStream_t stream)
{
    return resample_batch_at(plan, 0u, stream);
}

int rs_batch_log_mean_weight(const rs_batch_plan *plan, double *acc, hipStream_t stream)
{
    if (!plan || !plan->dev || plan->n_instances < 1 || !acc) return RS_EINVAL;
    const rs::BatchInstance *insts = static_cast<const rs::BatchInstance *>(plan->dev);
    const int rc = rs::launch_batch_log_mean_weight(insts, plan->n_instances, acc, stream);
    return rc == 0 ? RS_OK : RS_EHIP;
}

int rs_batch_iterations(const rs_batch_plan *plan, uint32_t *out, hipStream_t stream)
{
    if (!plan || !plan->dev || plan->n_instances < 1 || !out) return RS_EINVAL;
    const rs::BatchInstance *insts = static_cast<const rs::BatchInstance *>(plan->dev);
    const int rc = rs::launch_batch_iterations(insts, plan->n_instances, out, stream);
    return rc == 0 ? RS_OK : RS_EHIP;
}

int resample_batch_at(const rs_batch_plan *plan, uint32_t instance_add, hipStream_t stream)
{
    if (!plan || !plan->dev || plan->n_instances < 1) return RS_EINVAL;
    const unsigned char *base = static_cast<const unsigned char *>(plan->dev);
    rs::BatchLaunch L;
    L.insts = reinterpret_cast<const rs::BatchInstance *>(base);
    L.tile_items = reinterpret_cast<const int2 *>(base + plan->off_tile_items);
    L.table_items = reinterpret_cast<const int32_t *>(base + plan->off_table_items);
    L.main_items = reinterpret_cast<const int2 *>(base + plan->off_main_items);
    L.n_tile_items = plan->n_tile_items;
    L.n_table_items = plan->n_table_items;
    L.n_main_items = plan->n_main_items;
    L.blocks = plan->blocks;
    L.unroll = plan->unroll;
    L.chains_per_item = plan->chains_per_item;
    L.lds_max_p = plan->lds_max_p;
    L.max_table_tiles = plan->max_table_tiles;
    L.smem_main = (size_t)plan->smem_main;
    L.instance_add = instance_add;
    const int rc = rs::launch_batch(L, stream);
    return rc == 0 ? RS_OK : (rc == -1 ? RS_EINVAL : RS_EHIP);
}

}  // extern "C"
