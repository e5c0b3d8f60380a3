// Batched ensemble of independent lattices (include/lbm_axi_batch.h): one
// persistent launch per step over a work list of (instance, tile) items,
// replayed from a captured HIP graph, with a timing autotuner over the
// compiled tile configurations, the grid size and the work-list order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/lbm_axi.h"
#include "../../include/lbm_axi_batch.h"
#include "common.hpp"
#include "batch_kernel.hpp"

using namespace lbm_host;

namespace {

struct Config {
    int tz, tr, nt;
};
// compiled configurations per precision (index = configuration id)
constexpr Config kCfg32[] = {{64, 16, 256}, {64, 16, 512}, {128, 16, 512}, {64, 32, 512}, {32, 16, 512}};
constexpr Config kCfg64[] = {{64, 16, 512}, {64, 32, 512}, {64, 32, 1024}, {32, 16, 512}};
constexpr int kNCfg32 = 5, kNCfg64 = 4;

template <class P, int TZ, int TR, int NT, int kOpt>
void launch_batch_t(dim3 grid, hipStream_t s, const lbm::BatchInstance* insts, const int2* items, int n, int parity) {
    hipLaunchKernelGGL((lbm::axi_batch_kernel<P, TZ, TR, NT, kOpt>), grid, dim3(NT), 0, s, insts, items, n, parity);
}
template <class P, int TZ, int TR, int NT, bool kMoments, int kOpt>
void launch_tile_t(dim3 grid, hipStream_t s, const lbm::StepArgs& a) {
    hipLaunchKernelGGL((lbm::axi_tile_kernel<P, TZ, TR, NT, kMoments, kOpt>), grid, dim3(NT), 0, s, a);
}

using BatchFn = void (*)(dim3, hipStream_t, const lbm::BatchInstance*, const int2*, int, int);
using TileFn = void (*)(dim3, hipStream_t, const lbm::StepArgs&);

// [o]: 0 every instance with the default options; 1 some instance sets an
// option bit, which the kernels then read per instance at run time
#define LBM_CFG32(F, ...) {F<lbm::PrecF32S, 64, 16, 256, __VA_ARGS__>, F<lbm::PrecF32S, 64, 16, 512, __VA_ARGS__>, \
                           F<lbm::PrecF32S, 128, 16, 512, __VA_ARGS__>, F<lbm::PrecF32S, 64, 32, 512, __VA_ARGS__>, \
                           F<lbm::PrecF32S, 32, 16, 512, __VA_ARGS__>}
#define LBM_CFG64(F, ...) {F<lbm::PrecF64, 64, 16, 512, __VA_ARGS__>, F<lbm::PrecF64, 64, 32, 512, __VA_ARGS__>, \
                           F<lbm::PrecF64, 64, 32, 1024, __VA_ARGS__>, F<lbm::PrecF64, 32, 16, 512, __VA_ARGS__>}
constexpr BatchFn kBatch32[2][kNCfg32] = {LBM_CFG32(launch_batch_t, 0), LBM_CFG32(launch_batch_t, -1)};
constexpr BatchFn kBatch64[2][kNCfg64] = {LBM_CFG64(launch_batch_t, 0), LBM_CFG64(launch_batch_t, -1)};
constexpr TileFn kStep32[2][kNCfg32] = {LBM_CFG32(launch_tile_t, false, 0), LBM_CFG32(launch_tile_t, false, -1)};
constexpr TileFn kStep64[2][kNCfg64] = {LBM_CFG64(launch_tile_t, false, 0), LBM_CFG64(launch_tile_t, false, -1)};
constexpr TileFn kMom32[2][kNCfg32] = {LBM_CFG32(launch_tile_t, true, 0), LBM_CFG32(launch_tile_t, true, -1)};
constexpr TileFn kMom64[2][kNCfg64] = {LBM_CFG64(launch_tile_t, true, 0), LBM_CFG64(launch_tile_t, true, -1)};
#undef LBM_CFG32
#undef LBM_CFG64

int tiles_of(const lbm_axi_params& p, const Config& c) {
    return ((p.nz + c.tz - 1) / c.tz) * ((p.nr + c.tr - 1) / c.tr);
}

}  // namespace

struct lbm_axi_batch {
    std::vector<lbm_axi_params> p;
    std::vector<size_t> off[3];  // buffer 0, buffer 1, backup
    size_t state_bytes_max = 0;
    size_t off_tab = 0, off_items = 0;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int precision = 0;
    int parity = 0;
    int cfg = 0, grid_per_cu = 2, order = 1;
    int any_guo = 0;  // 1 if some instance sets an option bit (Guo forcing, wall derivatives, z walls)
    int n_items = 0, cus = 256;
    std::vector<lbm::BatchInstance> host_tab;
    hipGraphExec_t graph[2] = {nullptr, nullptr};

    const Config& config() const { return precision == LBM_AXI_FP64 ? kCfg64[cfg] : kCfg32[cfg]; }
    int n_cfg() const { return precision == LBM_AXI_FP64 ? kNCfg64 : kNCfg32; }
    // the caller's view of instance k's state: 9 nz nr values
    size_t state_bytes(int k) const { return 9 * (size_t)p[k].nz * p[k].nr * storage_size(precision); }
    // the instance's buffers pad each plane by kPlanePadBytes, as the
    // single-lattice library does (planes 2^k bytes apart share channels)
    long long pitch(int k) const {
        return (long long)p[k].nz * p[k].nr + kPlanePadBytes / (long long)storage_size(precision);
    }
    size_t buf_bytes(int k) const { return 9 * (size_t)pitch(k) * storage_size(precision); }
    void* buf(int k, int which) { return ws + off[which][k]; }
};

namespace {

size_t layout(const lbm_axi_params* ps, int32_t n, lbm_axi_batch* b) {
    size_t off = 0, items_max = 0;
    const int prec = ps[0].precision;
    for (int w = 0; w < 3; ++w) {
        for (int k = 0; k < n; ++k) {
            const size_t bytes =
                9 * ((size_t)ps[k].nz * ps[k].nr + (size_t)kPlanePadBytes / storage_size(prec)) * storage_size(prec);
            if (b) b->off[w].push_back(off);
            off += align_up(bytes);
        }
    }
    const int ncfg = prec == LBM_AXI_FP64 ? kNCfg64 : kNCfg32;
    for (int c = 0; c < ncfg; ++c) {
        size_t items = 0;
        for (int k = 0; k < n; ++k) items += tiles_of(ps[k], prec == LBM_AXI_FP64 ? kCfg64[c] : kCfg32[c]);
        items_max = std::max(items_max, items);
    }
    const size_t off_tab = off;
    off += align_up((size_t)n * sizeof(lbm::BatchInstance));
    const size_t off_items = off;
    off += align_up(items_max * sizeof(int2));
    if (b) {
        b->off_tab = off_tab;
        b->off_items = off_items;
    }
    return off;
}

int check_all(const lbm_axi_params* ps, int32_t n) {
    if (!ps || n < 1) return fail(LBM_AXI_EINVAL, "need at least one instance");
    for (int k = 0; k < n; ++k) {
        int rc = check_params(&ps[k]);
        if (rc != LBM_AXI_OK) return fail(rc, "instance %d: %s", k, g_last_error.c_str());
        if (ps[k].precision != ps[0].precision) return fail(LBM_AXI_EINVAL, "instance %d: precisions differ", k);
        if (ps[k].flags & LBM_AXI_FLAG_MIDLINK)
            return fail(LBM_AXI_EUNSUP, "instance %d: LBM_AXI_FLAG_MIDLINK is not supported in a batch", k);
    }
    return LBM_AXI_OK;
}

lbm::StepArgs instance_args(lbm_axi_batch* b, int k, int parity) {
    const lbm_axi_params& p = b->p[k];
    const Config& c = b->config();
    lbm::StepArgs a{};
    a.fin = b->buf(k, parity);
    a.fout = b->buf(k, 1 - parity);
    a.plane = b->pitch(k);
    a.state_bytes = (unsigned)b->buf_bytes(k);
    a.nz = p.nz;
    a.nr = p.nr;
    a.tiles_z = (p.nz + c.tz - 1) / c.tz;
    a.big_nz = p.nz >= c.tz + 6 ? 1 : 0;
    a.wall = p.wall;
    a.axisym = p.axisym;
    a.opts = lbm_host::option_bits(p.flags);
    a.G = p.G;
    a.tau = p.tau;
    a.rho0 = p.psi_rho0;
    a.gz = p.gz;
    a.rho_ref = b->precision == LBM_AXI_FP64 ? 0.0 : p.rho_ref;
    a.in_row = -1;  // batch instances have no open rows
    a.out_row = -1;
    return a;
}

void drop_graphs(lbm_axi_batch* b) {
    for (auto& g : b->graph) {
        if (g) (void)hipGraphExecDestroy(g);  // teardown: nothing to report
        g = nullptr;
    }
}

// rebuild the device instance table and the work list for the schedule
int rebuild(lbm_axi_batch* b) {
    drop_graphs(b);
    const int n = (int)b->p.size();
    const Config& c = b->config();
    b->host_tab.resize(n);
    for (int k = 0; k < n; ++k) {
        b->host_tab[k].args[0] = instance_args(b, k, 0);
        b->host_tab[k].args[1] = instance_args(b, k, 1);
    }
    std::vector<int> inst(n);
    std::iota(inst.begin(), inst.end(), 0);
    if (b->order == 1)
        std::stable_sort(inst.begin(), inst.end(), [&](int x, int y) {
            return (long long)b->p[x].nz * b->p[x].nr > (long long)b->p[y].nz * b->p[y].nr;
        });
    std::vector<int2> items;
    if (b->order == 2) {
        int maxt = 0;
        for (int k = 0; k < n; ++k) maxt = std::max(maxt, tiles_of(b->p[k], c));
        for (int t = 0; t < maxt; ++t)
            for (int k : inst)
                if (t < tiles_of(b->p[k], c)) items.push_back(make_int2(k, t));
    } else {
        for (int k : inst)
            for (int t = 0; t < tiles_of(b->p[k], c); ++t) items.push_back(make_int2(k, t));
    }
    b->n_items = (int)items.size();
    // launches already queued may still read the current tables
    HIP_TRY(hipStreamSynchronize(b->stream), "batch synchronize before table upload");
    HIP_TRY(hipMemcpy(b->ws + b->off_tab, b->host_tab.data(), n * sizeof(lbm::BatchInstance), hipMemcpyHostToDevice),
            "batch table upload");
    HIP_TRY(hipMemcpy(b->ws + b->off_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice),
            "batch work list upload");
    return LBM_AXI_OK;
}

// a multiple of 8 workgroups, at least 8: the batch kernel splits the work
// list into one contiguous range per XCD
int grid_size(lbm_axi_batch* b) {
    const int g = std::max(1, std::min(b->n_items, b->grid_per_cu * b->cus));
    return (g + 7) / 8 * 8;
}

int launch_once(lbm_axi_batch* b, hipStream_t s, int parity) {
    const BatchFn fn = b->precision == LBM_AXI_FP64 ? kBatch64[b->any_guo][b->cfg] : kBatch32[b->any_guo][b->cfg];
    fn(dim3(grid_size(b)), s, reinterpret_cast<const lbm::BatchInstance*>(b->ws + b->off_tab),
       reinterpret_cast<const int2*>(b->ws + b->off_items), b->n_items, parity);
    HIP_TRY(hipGetLastError(), "batch kernel launch");
    return LBM_AXI_OK;
}

int ensure_graph(lbm_axi_batch* b, int parity) {
    if (b->graph[parity]) return LBM_AXI_OK;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "graph capture begin");
    int rc = launch_once(b, b->stream, parity);
    if (rc == LBM_AXI_OK) rc = launch_once(b, b->stream, 1 - parity);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc != LBM_AXI_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "graph capture end");
    e = hipGraphInstantiate(&b->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the executable graph keeps what it needs
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    return LBM_AXI_OK;
}

int copy_states(lbm_axi_batch* b, int from, int to) {
    for (size_t k = 0; k < b->p.size(); ++k)
        HIP_TRY(hipMemcpyAsync(b->buf((int)k, to), b->buf((int)k, from), b->buf_bytes((int)k),
                               hipMemcpyDeviceToDevice, b->stream),
                "batch state copy");
    return LBM_AXI_OK;
}

}  // namespace

extern "C" {

size_t lbm_axi_batch_workspace_bytes(const lbm_axi_params* ps, int32_t n_inst) {
    if (check_all(ps, n_inst) != LBM_AXI_OK) return 0;
    return layout(ps, n_inst, nullptr);
}

int lbm_axi_batch_create(const lbm_axi_params* ps, int32_t n_inst, const double* const* h_d_rho0, void* d_workspace,
                         size_t ws_bytes, void* hip_stream, lbm_axi_batch_t* out) {
    int rc = check_all(ps, n_inst);
    if (rc != LBM_AXI_OK) return rc;
    if (!out || !h_d_rho0 || !d_workspace) return fail(LBM_AXI_EINVAL, "NULL argument");
    *out = nullptr;
    if ((uintptr_t)d_workspace % kAlign) return fail(LBM_AXI_EINVAL, "workspace must be 256-byte aligned");
    for (int k = 0; k < n_inst; ++k)
        if (!h_d_rho0[k]) return fail(LBM_AXI_EINVAL, "rho0 of instance %d is NULL", k);
    const size_t need = layout(ps, n_inst, nullptr);
    if (ws_bytes < need) return fail(LBM_AXI_ENOMEM, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    auto* b = new (std::nothrow) lbm_axi_batch();
    if (!b) return fail(LBM_AXI_ENOMEM, "host allocation failed");
    b->p.assign(ps, ps + n_inst);
    layout(ps, n_inst, b);
    b->ws = static_cast<char*>(d_workspace);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->precision = ps[0].precision;
    for (int k = 0; k < n_inst; ++k)
        if (ps[k].flags != 0) b->any_guo = 1;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "get device");
    if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->cus < 1)
        b->cus = 256;
    b->cfg = b->precision == LBM_AXI_FP64 ? 3 : 4;  // 32 x 16 tiles, as for a single small lattice, until tuned
    for (int k = 0; k < n_inst; ++k) {
        const long long n = (long long)ps[k].nz * ps[k].nr;
        const int blocks = (int)((n + 255) / 256);
        if (b->precision == LBM_AXI_FP64)
            hipLaunchKernelGGL(init_equilibrium_kernel<lbm::PrecF64>, dim3(blocks), dim3(256), 0, b->stream,
                               static_cast<double*>(b->buf(k, 0)), h_d_rho0[k], nullptr, nullptr, n, b->pitch(k), 0.0);
        else
            hipLaunchKernelGGL(init_equilibrium_kernel<lbm::PrecF32S>, dim3(blocks), dim3(256), 0, b->stream,
                               static_cast<float*>(b->buf(k, 0)), h_d_rho0[k], nullptr, nullptr, n, b->pitch(k), ps[k].rho_ref);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch init launch");
    }
    rc = rebuild(b);
    if (rc != LBM_AXI_OK) {
        delete b;
        return rc;
    }
    *out = b;
    for (int k = 0; k < n_inst; ++k)
        if (ps[k].G < -6.0) return stability_warning(ps[k].G);
    return LBM_AXI_OK;
}

int lbm_axi_batch_step(lbm_axi_batch_t b, int64_t n) {
    if (!b) return fail(LBM_AXI_EINVAL, "batch is NULL");
    if (n < 0) return fail(LBM_AXI_EINVAL, "n must be >= 0");
    // a stream the caller is capturing into a graph of its own gets the
    // launches themselves; the buffer parity is host state, so a capture
    // that is to be replayed must hold an even number of steps
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (b->stream != nullptr) HIP_TRY(hipStreamIsCapturing(b->stream, &cs), "stream capture status");
    const bool captured = cs != hipStreamCaptureStatusNone;
    if (captured && (n & 1))
        return fail(LBM_AXI_EINVAL, "n must be even while the stream is being captured (got %lld)", (long long)n);
    const bool graphs = b->stream != nullptr && !captured;
    int64_t done = 0;
    if (graphs && n >= 2) {
        int rc = ensure_graph(b, b->parity);
        if (rc != LBM_AXI_OK) return rc;
        for (; done + 2 <= n; done += 2) HIP_TRY(hipGraphLaunch(b->graph[b->parity], b->stream), "graph launch");
    }
    for (; done < n; ++done) {
        int rc = launch_once(b, b->stream, b->parity);
        if (rc != LBM_AXI_OK) return rc;
        b->parity = 1 - b->parity;
    }
    return LBM_AXI_OK;
}

int lbm_axi_batch_step_per_instance(lbm_axi_batch_t b, int64_t n) {
    if (!b) return fail(LBM_AXI_EINVAL, "batch is NULL");
    if (n < 0) return fail(LBM_AXI_EINVAL, "n must be >= 0");
    const TileFn fn = b->precision == LBM_AXI_FP64 ? kStep64[b->any_guo][b->cfg] : kStep32[b->any_guo][b->cfg];
    for (int64_t s = 0; s < n; ++s) {
        for (size_t k = 0; k < b->p.size(); ++k)
            fn(dim3(tiles_of(b->p[k], b->config())), b->stream, b->host_tab[k].args[b->parity]);
        HIP_TRY(hipGetLastError(), "per-instance launch");
        b->parity = 1 - b->parity;
    }
    return LBM_AXI_OK;
}

int lbm_axi_batch_moments(lbm_axi_batch_t b, int32_t k, double* d_rho, double* d_uz, double* d_ur) {
    if (!b || k < 0 || k >= (int)b->p.size()) return fail(LBM_AXI_EINVAL, "bad batch or instance");
    lbm::StepArgs a = b->host_tab[k].args[b->parity];
    a.rho_out = d_rho;
    a.uz_out = d_uz;
    a.ur_out = d_ur;
    a.partials = nullptr;
    const TileFn fn = b->precision == LBM_AXI_FP64 ? kMom64[b->any_guo][b->cfg] : kMom32[b->any_guo][b->cfg];
    fn(dim3(tiles_of(b->p[k], b->config())), b->stream, a);
    HIP_TRY(hipGetLastError(), "moments launch");
    return LBM_AXI_OK;
}

int lbm_axi_batch_populations(lbm_axi_batch_t b, int32_t k, double* d_f) {
    if (!b || k < 0 || k >= (int)b->p.size() || !d_f) return fail(LBM_AXI_EINVAL, "bad batch, instance or d_f");
    const lbm_axi_params& q = b->p[k];
    const long long n = (long long)q.nz * q.nr;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (b->precision == LBM_AXI_FP64)
        hipLaunchKernelGGL(decode_populations_kernel<lbm::PrecF64>, grid, dim3(256), 0, b->stream,
                           static_cast<const double*>(b->buf(k, b->parity)), b->pitch(k), n, 0.0, d_f);
    else
        hipLaunchKernelGGL(decode_populations_kernel<lbm::PrecF32S>, grid, dim3(256), 0, b->stream,
                           static_cast<const float*>(b->buf(k, b->parity)), b->pitch(k), n, q.rho_ref, d_f);
    HIP_TRY(hipGetLastError(), "populations kernel launch");
    return LBM_AXI_OK;
}

int lbm_axi_batch_get_state(lbm_axi_batch_t b, int32_t k, void* d_dst) {
    if (!b || k < 0 || k >= (int)b->p.size() || !d_dst) return fail(LBM_AXI_EINVAL, "bad batch, instance or dst");
    const size_t row = b->state_bytes(k) / 9, padded = b->buf_bytes(k) / 9;
    HIP_TRY(hipMemcpy2DAsync(d_dst, row, b->buf(k, b->parity), padded, row, 9, hipMemcpyDeviceToDevice, b->stream),
            "get_state copy");
    return LBM_AXI_OK;
}

int32_t lbm_axi_batch_num_configs(lbm_axi_batch_t b) { return b ? b->n_cfg() : 0; }

int lbm_axi_batch_config_info(lbm_axi_batch_t b, int32_t c, int32_t* h_tz, int32_t* h_tr, int32_t* h_threads) {
    if (!b || c < 0 || c >= b->n_cfg()) return fail(LBM_AXI_EINVAL, "bad configuration");
    const Config& x = b->precision == LBM_AXI_FP64 ? kCfg64[c] : kCfg32[c];
    if (h_tz) *h_tz = x.tz;
    if (h_tr) *h_tr = x.tr;
    if (h_threads) *h_threads = x.nt;
    return LBM_AXI_OK;
}

int lbm_axi_batch_set_schedule(lbm_axi_batch_t b, int32_t c, int32_t grid_per_cu, int32_t order) {
    if (!b || c < 0 || c >= b->n_cfg() || grid_per_cu < 1 || grid_per_cu > 64 || order < 0 || order > 2)
        return fail(LBM_AXI_EINVAL, "bad schedule");
    b->cfg = c;
    b->grid_per_cu = grid_per_cu;
    b->order = order;
    return rebuild(b);
}

int lbm_axi_batch_autotune(lbm_axi_batch_t b, int32_t steps_per_trial, int32_t* h_choice, double* h_us) {
    if (!b || steps_per_trial < 1) return fail(LBM_AXI_EINVAL, "bad autotune arguments");
    int rc = copy_states(b, b->parity, 2);  // backup
    if (rc != LBM_AXI_OK) return rc;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    double best = 1e300;
    int bc = b->cfg, bg = b->grid_per_cu, bo = b->order;
    for (int c = 0; c < b->n_cfg() && rc == LBM_AXI_OK; ++c)
        for (int g = 1; g <= 4 && rc == LBM_AXI_OK; ++g)
            for (int o = 0; o <= 2 && rc == LBM_AXI_OK; ++o) {
                b->cfg = c;
                b->grid_per_cu = g;
                b->order = o;
                if ((rc = rebuild(b)) != LBM_AXI_OK) break;
                if ((rc = launch_once(b, b->stream, b->parity)) != LBM_AXI_OK) break;  // warm-up
                b->parity = 1 - b->parity;
                if (hipEventRecord(e0, b->stream) != hipSuccess) {
                    rc = fail(LBM_AXI_EHIP, "autotune event record");
                    break;
                }
                for (int s = 0; s < steps_per_trial && rc == LBM_AXI_OK; ++s) {
                    rc = launch_once(b, b->stream, b->parity);
                    b->parity = 1 - b->parity;
                }
                if (rc != LBM_AXI_OK) break;
                float ms = 0.f;
                if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = fail(LBM_AXI_EHIP, "autotune timing");
                    break;
                }
                const double us = 1000.0 * ms / steps_per_trial;
                if (us < best) {
                    best = us;
                    bc = c;
                    bg = g;
                    bo = o;
                }
                // restore the populations
                if ((rc = copy_states(b, 2, b->parity)) != LBM_AXI_OK) break;
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_AXI_OK) return rc;
    b->cfg = bc;
    b->grid_per_cu = bg;
    b->order = bo;
    rc = rebuild(b);
    if (rc != LBM_AXI_OK) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream), "autotune finish");
    if (h_choice) {
        h_choice[0] = bc;
        h_choice[1] = bg;
        h_choice[2] = bo;
    }
    if (h_us) *h_us = best;
    return LBM_AXI_OK;
}

int64_t lbm_axi_batch_nodes(lbm_axi_batch_t b) {
    if (!b) return 0;
    int64_t s = 0;
    for (const auto& p : b->p) s += (int64_t)p.nz * p.nr;
    return s;
}

void lbm_axi_batch_destroy(lbm_axi_batch_t b) {
    if (!b) return;
    drop_graphs(b);
    delete b;
}

}  // extern "C"
