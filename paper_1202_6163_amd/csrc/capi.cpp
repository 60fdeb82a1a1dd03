// C ABI of the resampling library: argument checking, workspace sizing,
// Metropolis launch tuning and the host-side iteration-count helper. Every
// check here happens before any kernel is enqueued.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

#include "analysis.h"
#include "launch.h"
#include "prefix.h"
#include "resample.h"

namespace {
thread_local hipError_t g_last_hip_error = hipSuccess;
}  // namespace

namespace rs {
int record_hip_error(hipError_t e)
{
    if (e == hipSuccess) return 0;
    g_last_hip_error = e;
    return -3;
}
int launch_status() { return record_hip_error(hipGetLastError()); }

int allow_dynamic_lds(const void *fn, size_t bytes)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, size_t> granted;  // (device, kernel) -> bytes
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return record_hip_error(e);
    std::lock_guard<std::mutex> lock(mu);
    size_t &have = granted[{dev, fn}];
    if (bytes <= have) return 0;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return record_hip_error(e);
    have = bytes;
    return 0;
}
}  // namespace rs

namespace {

constexpr int64_t kMaxP = 2147483647;  // ancestors are int32

// P rows of D binary32 values are at most 2^40 values (4 TiB), so byte
// counts and element indices never overflow; callers have checked P >= 1.
bool state_too_big(int64_t P, int32_t D) { return (size_t)D > ((size_t)1 << 40) / (size_t)P; }

std::mutex g_tune_mutex;
bool g_tune_init = false;
rs::MetropolisTuning g_tune{256, 8, 16384, 0};

bool valid_tuning(const rs::MetropolisTuning &t)
{
    const bool lpc_ok = t.lanes_per_chain == 0 ||
                        (t.lanes_per_chain >= 1 && t.lanes_per_chain <= 64 &&
                         (t.lanes_per_chain & (t.lanes_per_chain - 1)) == 0);
    const bool unroll_ok = t.unroll == 2 || t.unroll == 4 || t.unroll == 8 || t.unroll == 16;
    return t.block >= 64 && t.block <= 1024 && t.block % 64 == 0 && unroll_ok &&
           t.lds_max_p >= 0 && lpc_ok;
}

long env_long(const char *name, long fallback)
{
    const char *s = std::getenv(name);
    if (!s || !*s) return fallback;
    char *end = nullptr;
    const long v = std::strtol(s, &end, 10);
    return (end && *end == '\0') ? v : fallback;
}

// Environment overrides pick launch parameters only, never another code path.
rs::MetropolisTuning current_tuning()
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    if (!g_tune_init) {
        rs::MetropolisTuning t = g_tune;
        t.block = (int32_t)env_long("RS_BLOCK", t.block);
        t.unroll = (int32_t)env_long("RS_UNROLL", t.unroll);
        t.lds_max_p = (int64_t)env_long("RS_LDS_MAX_P", (long)t.lds_max_p);
        t.lanes_per_chain = (int32_t)env_long("RS_LANES_PER_CHAIN", t.lanes_per_chain);
        if (valid_tuning(t)) g_tune = t;
        g_tune_init = true;
    }
    return g_tune;
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Workspace sections start 256 bytes apart and are read with 16-byte vector
// loads, so the workspace itself must start on a 256-byte boundary (as
// hipMalloc's blocks do).
bool misaligned(const void *ws) { return ((uintptr_t)ws & 255u) != 0; }

int map_rc(int rc) { return rc == 0 ? RS_OK : (rc == -1 ? RS_EINVAL : RS_EHIP); }

int prefix_call(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                uint32_t instance, double *cumw, void *ws, size_t ws_bytes, int32_t *status,
                hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!lw || (!anc && !off) || !ws || misaligned(ws) || P < 0 || P > kMaxP) return RS_EINVAL;
    if (off && kind == rs::kMultinomial) return RS_EINVAL;
    const size_t p = (size_t)P;
    const void *outs[3] = {anc, off, cumw};
    const size_t out_bytes[3] = {4 * p, 4 * p, 8 * p};
    for (int a = 0; a < 3; ++a) {
        if (!outs[a]) continue;
        if (overlaps(outs[a], out_bytes[a], lw, 4 * p)) return RS_EINVAL;
        for (int b = a + 1; b < 3; ++b)
            if (outs[b] && overlaps(outs[a], out_bytes[a], outs[b], out_bytes[b])) return RS_EINVAL;
    }
    if (ws_bytes < rs_workspace_bytes(P, kind)) return RS_EWORKSPACE;
    if (overlaps(ws, ws_bytes, lw, 4 * p)) return RS_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (outs[a] && overlaps(ws, ws_bytes, outs[a], out_bytes[a])) return RS_EINVAL;
    return map_rc(
        rs::launch_prefix(kind, lw, anc, off, P, seed, instance, cumw, ws, status, stream));
}

}  // namespace

extern "C" {

const char *rs_strerror(int code)
{
    switch (code) {
    case RS_OK: return "success";
    case RS_EINVAL: return "invalid argument";
    case RS_EWORKSPACE: return "workspace too small";
    case RS_EHIP: return "HIP launch failure";
    default: return "unknown error";
    }
}

int rs_version(void) { return 100; }

const char *rs_last_hip_error(void) { return hipGetErrorString(g_last_hip_error); }

size_t rs_workspace_bytes(int64_t P, int resampler)
{
    if (P < 1) return 0;
    switch (resampler) {
    case RS_STRATIFIED:
    case RS_SYSTEMATIC:
    case RS_LOG_SUM_EXP:
    case RS_METROPOLIS_ADAPTIVE: return rs::ws_layout(P, false).total;
    case RS_MULTINOMIAL: return rs::ws_layout(P, true).total;
    default: return 0;
    }
}

int rs_workspace_init(void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (ws_bytes == 0) return RS_OK;
    if (!ws) return RS_EINVAL;
    return map_rc(rs::launch_zero(ws, ws_bytes, stream));
}

int resample_metropolis(const float *lw, int32_t *anc, int64_t P, uint32_t B, uint64_t seed,
                        uint32_t instance, int32_t *status, hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!lw || !anc || P < 0 || P > kMaxP) return RS_EINVAL;
    if (overlaps(lw, 4 * (size_t)P, anc, 4 * (size_t)P)) return RS_EINVAL;
    const rs::MetropolisTuning t = current_tuning();
    return map_rc(rs::launch_metropolis(lw, anc, P, B, seed, instance, status, t, stream));
}

int resample_stratified(const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                        uint32_t instance, double *cumw, void *ws, size_t ws_bytes,
                        int32_t *status, hipStream_t stream)
{
    return prefix_call(RS_STRATIFIED, lw, anc, off, P, seed, instance, cumw, ws, ws_bytes, status,
                       stream);
}

int resample_systematic(const float *lw, int32_t *anc, int32_t *off, int64_t P, uint64_t seed,
                        uint32_t instance, double *cumw, void *ws, size_t ws_bytes,
                        int32_t *status, hipStream_t stream)
{
    return prefix_call(RS_SYSTEMATIC, lw, anc, off, P, seed, instance, cumw, ws, ws_bytes, status,
                       stream);
}

int resample_prefix_static(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P,
                           uint64_t seed, uint32_t instance, double *cumw, int32_t *status,
                           hipStream_t stream)
{
    if (kind != RS_STRATIFIED && kind != RS_SYSTEMATIC && kind != RS_MULTINOMIAL)
        return RS_EINVAL;
    if (P == 0) return RS_OK;
    if (P < 0 || P > kMaxP) return RS_EINVAL;
    if (rs_workspace_bytes(P, kind) > RS_STATIC_SCRATCH_BYTES) return RS_EWORKSPACE;
    void *ws = nullptr;
    const int rc = rs::static_scratch(&ws);
    if (rc) return map_rc(rc);
    return prefix_call(kind, lw, anc, off, P, seed, instance, cumw, ws, RS_STATIC_SCRATCH_BYTES,
                       status, stream);
}

int resample_multinomial(const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                         uint32_t instance, double *cumw, void *ws, size_t ws_bytes,
                         int32_t *status, hipStream_t stream)
{
    return prefix_call(RS_MULTINOMIAL, lw, anc, nullptr, P, seed, instance, cumw, ws, ws_bytes,
                       status, stream);
}

int resample_and_copy(int kind, const float *lw, int32_t *anc, int32_t *off, int64_t P, uint32_t B,
                      uint64_t seed, uint32_t instance, const float *x_in, float *x_out,
                      int32_t D, void *ws, size_t ws_bytes, int32_t *status, hipStream_t stream)
{
    const bool prefix = kind == RS_STRATIFIED || kind == RS_SYSTEMATIC || kind == RS_MULTINOMIAL;
    if (!prefix && kind != RS_METROPOLIS) return RS_EINVAL;
    if (P == 0) return RS_OK;
    if (!lw || !anc || !x_in || !x_out || D < 1 || P < 0 || P > kMaxP) return RS_EINVAL;
    if (off && kind != RS_STRATIFIED && kind != RS_SYSTEMATIC) return RS_EINVAL;
    if (state_too_big(P, D)) return RS_EINVAL;
    const size_t p = (size_t)P, rows = p * (size_t)D * sizeof(float);
    // written: anc, off, x_out; read: lw, x_in
    const void *outs[3] = {anc, off, x_out};
    const size_t out_bytes[3] = {4 * p, 4 * p, rows};
    for (int a = 0; a < 3; ++a) {
        if (!outs[a]) continue;
        if (overlaps(outs[a], out_bytes[a], lw, 4 * p) || overlaps(outs[a], out_bytes[a], x_in, rows))
            return RS_EINVAL;
        for (int b = a + 1; b < 3; ++b)
            if (outs[b] && overlaps(outs[a], out_bytes[a], outs[b], out_bytes[b])) return RS_EINVAL;
    }
    rs::Rows r;
    r.x_in = x_in;
    r.x_out = x_out;
    r.D = D;
    if (kind == RS_METROPOLIS) {
        const rs::MetropolisTuning t = current_tuning();
        return map_rc(rs::launch_metropolis(lw, anc, P, B, seed, instance, status, t, stream, r));
    }
    if (!ws || misaligned(ws)) return RS_EINVAL;
    if (ws_bytes < rs_workspace_bytes(P, kind)) return RS_EWORKSPACE;
    if (overlaps(ws, ws_bytes, lw, 4 * p) || overlaps(ws, ws_bytes, x_in, rows)) return RS_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (outs[a] && overlaps(ws, ws_bytes, outs[a], out_bytes[a])) return RS_EINVAL;
    return map_rc(rs::launch_prefix(kind, lw, anc, off, P, seed, instance, nullptr, ws, status,
                                    stream, r));
}

int rs_workspace_log_sum_exp(const void *ws, int64_t P, double *out, hipStream_t stream)
{
    if (!ws || misaligned(ws) || !out || P < 1 || P > kMaxP) return RS_EINVAL;
    return map_rc(rs::launch_workspace_lse(ws, P, out, stream));
}

size_t rs_sorted_workspace_bytes(int64_t P, int kind)
{
    if (P < 1 || (kind != RS_STRATIFIED && kind != RS_SYSTEMATIC && kind != RS_MULTINOMIAL))
        return 0;
    return rs::sorted_layout(P, kind).total;
}

int resample_sorted(int kind, const float *lw, int32_t *anc, int64_t P, uint64_t seed,
                    uint32_t instance, void *ws, size_t ws_bytes, int32_t *status,
                    hipStream_t stream)
{
    if (kind != RS_STRATIFIED && kind != RS_SYSTEMATIC && kind != RS_MULTINOMIAL) return RS_EINVAL;
    if (P == 0) return RS_OK;
    if (!lw || !anc || !ws || misaligned(ws) || P < 0 || P > kMaxP) return RS_EINVAL;
    const size_t p = (size_t)P;
    if (overlaps(lw, 4 * p, anc, 4 * p)) return RS_EINVAL;
    if (ws_bytes < rs_sorted_workspace_bytes(P, kind)) return RS_EWORKSPACE;
    if (overlaps(ws, ws_bytes, lw, 4 * p) || overlaps(ws, ws_bytes, anc, 4 * p)) return RS_EINVAL;
    return map_rc(rs::launch_sorted(kind, lw, anc, P, seed, instance, ws, status, stream));
}

int ancestors_to_offspring(const int32_t *anc, int32_t *off, int64_t P, int32_t *status,
                           hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!anc || !off || P < 0 || P > kMaxP) return RS_EINVAL;
    if (overlaps(anc, 4 * (size_t)P, off, 4 * (size_t)P)) return RS_EINVAL;
    return map_rc(rs::launch_offspring(anc, off, P, status, stream));
}

size_t rs_offspring_workspace_bytes(int64_t P) { return rs::offspring_workspace_bytes(P); }

int ancestors_to_offspring_ws(const int32_t *anc, int32_t *off, int64_t P, void *ws,
                              size_t ws_bytes, int32_t *status, hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!anc || !off || P < 0 || P > kMaxP) return RS_EINVAL;
    const size_t p4 = 4 * (size_t)P, need = rs_offspring_workspace_bytes(P);
    if (overlaps(anc, p4, off, p4)) return RS_EINVAL;
    if (need > 0) {
        if (!ws || misaligned(ws)) return RS_EINVAL;
        if (ws_bytes < need) return RS_EWORKSPACE;
        if (overlaps(ws, ws_bytes, anc, p4) || overlaps(ws, ws_bytes, off, p4)) return RS_EINVAL;
    }
    return map_rc(rs::launch_offspring_ws(anc, off, P, ws, status, stream));
}

int permute_copy(const int32_t *anc, const float *x_in, float *x_out, int64_t P, int32_t D,
                 int32_t *status, hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!anc || !x_in || !x_out || P < 0 || P > kMaxP || D < 1 || state_too_big(P, D))
        return RS_EINVAL;
    const size_t rows = (size_t)P * (size_t)D * sizeof(float);
    if (overlaps(x_in, rows, x_out, rows) || overlaps(anc, 4 * (size_t)P, x_out, rows))
        return RS_EINVAL;
    return map_rc(rs::launch_permute_copy(anc, x_in, x_out, P, D, status, stream));
}

size_t rs_inplace_workspace_bytes(int64_t P)
{
    return P < 1 ? 0 : rs::inplace_workspace_bytes(P);
}

int offspring_update_inplace(const int32_t *off, float *x, int64_t P, int32_t D, int32_t *anc,
                             void *ws, size_t ws_bytes, int32_t *status, hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!off || !x || !ws || misaligned(ws) || P < 0 || P > kMaxP || D < 1 ||
        state_too_big(P, D))
        return RS_EINVAL;
    const size_t rows = (size_t)P * (size_t)D * sizeof(float), p4 = 4 * (size_t)P;
    if (overlaps(off, p4, x, rows)) return RS_EINVAL;
    if (anc && (overlaps(anc, p4, off, p4) || overlaps(anc, p4, x, rows))) return RS_EINVAL;
    if (ws_bytes < rs_inplace_workspace_bytes(P)) return RS_EWORKSPACE;
    if (overlaps(ws, ws_bytes, off, p4) || overlaps(ws, ws_bytes, x, rows) ||
        (anc && overlaps(ws, ws_bytes, anc, p4)))
        return RS_EINVAL;
    return map_rc(rs::launch_offspring_update_inplace(off, x, P, D, anc, ws, status, stream));
}

int rs_log_sum_exp(const float *lw, int64_t P, double *out, void *ws, size_t ws_bytes,
                   int32_t *status, hipStream_t stream)
{
    if (!lw || !out || !ws || misaligned(ws) || P < 1 || P > kMaxP) return RS_EINVAL;
    if (ws_bytes < rs_workspace_bytes(P, RS_LOG_SUM_EXP)) return RS_EWORKSPACE;
    return map_rc(rs::launch_log_sum_exp(lw, P, out, ws, status, stream));
}

uint32_t metropolis_B(int64_t P, double w_max, double eps)
{
    return rs::iterations_for(P, w_max, eps);
}

int resample_metropolis_adaptive(const float *lw, int32_t *anc, int64_t P, double eps,
                                 uint32_t B_max, uint64_t seed, uint32_t instance, void *ws,
                                 size_t ws_bytes, uint32_t *B_used, int32_t *status,
                                 hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!lw || !anc || !ws || misaligned(ws) || P < 0 || P > kMaxP || !(eps > 0.0))
        return RS_EINVAL;
    if (overlaps(lw, 4 * (size_t)P, anc, 4 * (size_t)P)) return RS_EINVAL;
    if (ws_bytes < rs_workspace_bytes(P, RS_METROPOLIS_ADAPTIVE)) return RS_EWORKSPACE;
    if (overlaps(ws, ws_bytes, lw, 4 * (size_t)P) || overlaps(ws, ws_bytes, anc, 4 * (size_t)P))
        return RS_EINVAL;
    const rs::MetropolisTuning t = current_tuning();
    return map_rc(rs::launch_metropolis_adaptive(lw, anc, P, eps, B_max, seed, instance, ws,
                                                 B_used, status, t, stream));
}

int filter_loglik(const double *lse, int32_t T, int64_t P, double *out, hipStream_t stream)
{
    if (!lse || !out || T < 0 || P < 1 || P > kMaxP) return RS_EINVAL;
    if (overlaps(lse, 8 * (size_t)T, out, 8)) return RS_EINVAL;
    return map_rc(rs::launch_filter_loglik(lse, T, P, out, stream));
}

int filter_init(float *x, int64_t P, int32_t D, uint64_t seed, hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!x || P < 0 || P > kMaxP || D < 1 || D > 64) return RS_EINVAL;
    return map_rc(rs::launch_filter_init(x, P, 1, D, seed, stream));
}

int filter_init_batch(float *x, int32_t K, int64_t P, int32_t D, uint64_t seed,
                      hipStream_t stream)
{
    if (P == 0 || K == 0) return RS_OK;
    if (!x || K < 0 || P < 0 || P > kMaxP || D < 1 || D > 64) return RS_EINVAL;
    if ((int64_t)K * P > ((int64_t)1 << 40) / D) return RS_EINVAL;
    return map_rc(rs::launch_filter_init(x, P, K, D, seed, stream));
}

int filter_propagate_weight(const float *x_in, float *x_out, float *lw, int64_t P, int32_t D,
                            const double *A, const float *y, double q, double r, uint64_t seed,
                            uint32_t t, hipStream_t stream)
{
    if (P == 0) return RS_OK;
    if (!x_in || !x_out || !lw || !A || !y || P < 0 || P > kMaxP || D < 1 || D > 64)
        return RS_EINVAL;
    if (!(q >= 0.0) || !(r > 0.0)) return RS_EINVAL;
    const size_t rows = (size_t)P * (size_t)D * sizeof(float);
    if (overlaps(x_in, rows, x_out, rows) || overlaps(lw, 4 * (size_t)P, x_out, rows) ||
        overlaps(lw, 4 * (size_t)P, x_in, rows))
        return RS_EINVAL;
    return map_rc(
        rs::launch_filter_step(x_in, x_out, lw, P, 1, D, A, y, q, nullptr, r, seed, t, stream));
}

int filter_propagate_weight_batch(const float *x_in, float *x_out, float *lw, int32_t K, int64_t P,
                                  int32_t D, const double *A, const float *y, const double *q,
                                  double r, uint64_t seed, uint32_t t, hipStream_t stream)
{
    if (P == 0 || K == 0) return RS_OK;
    if (!x_in || !x_out || !lw || !A || !y || !q || K < 0 || P < 0 || P > kMaxP || D < 1 ||
        D > 64)
        return RS_EINVAL;
    if ((int64_t)K * P > ((int64_t)1 << 40) / D) return RS_EINVAL;
    if (!(r > 0.0)) return RS_EINVAL;
    const size_t n = (size_t)K * (size_t)P, rows = n * (size_t)D * sizeof(float);
    if (overlaps(x_in, rows, x_out, rows) || overlaps(lw, 4 * n, x_out, rows) ||
        overlaps(lw, 4 * n, x_in, rows))
        return RS_EINVAL;
    return map_rc(
        rs::launch_filter_step(x_in, x_out, lw, P, K, D, A, y, 0.0, q, r, seed, t, stream));
}

int rs_log_u_table(float *approx, float *exact, hipStream_t stream)
{
    if (!approx && !exact) return RS_EINVAL;
    if (approx && exact && overlaps(approx, 4u << 23, exact, 4u << 23)) return RS_EINVAL;
    return map_rc(rs::launch_log_u_table(approx, exact, stream));
}

int rs_probe_gather(const float *w, int64_t n, int64_t threads, int64_t rounds, uint32_t salt,
                    float *out, hipStream_t stream)
{
    if (!w || !out || n < 1 || n > kMaxP || threads < 256 || threads % 256 ||
        threads > (int64_t)1 << 30 || rounds < 1 || rounds > (int64_t)1 << 20)
        return RS_EINVAL;
    return map_rc(rs::launch_gather_probe(w, (uint32_t)n, (uint32_t)threads, (uint32_t)rounds, salt,
                                          out, stream));
}

int rs_probe_philox(uint64_t seed, int64_t threads, int64_t rounds, uint32_t *out,
                    hipStream_t stream)
{
    if (!out || threads < 256 || threads % 256 || threads > (int64_t)1 << 30 || rounds < 1 ||
        rounds > (int64_t)1 << 20)
        return RS_EINVAL;
    return map_rc(rs::launch_philox_probe(seed, (uint32_t)threads, (uint32_t)rounds, out, stream));
}

int rs_prefix_set_path(int path, int64_t wait_ns)
{
    return rs::set_prefix_path(path, wait_ns) == 0 ? RS_OK : RS_EINVAL;
}

int rs_prefix_get_path(void) { return rs::get_prefix_path(); }

int rs_metropolis_set_tuning(const rs_metropolis_tuning *t)
{
    if (!t) return RS_EINVAL;
    const rs::MetropolisTuning v{t->block, t->unroll, t->lds_max_p, t->lanes_per_chain};
    if (!valid_tuning(v)) return RS_EINVAL;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune = v;
    g_tune_init = true;
    return RS_OK;
}

int rs_metropolis_get_tuning(rs_metropolis_tuning *t)
{
    if (!t) return RS_EINVAL;
    const rs::MetropolisTuning v = current_tuning();
    t->block = v.block;
    t->unroll = v.unroll;
    t->lds_max_p = v.lds_max_p;
    t->lanes_per_chain = v.lanes_per_chain;
    return RS_OK;
}

}  // extern "C"
