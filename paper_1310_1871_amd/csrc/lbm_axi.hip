// C ABI of the axisymmetric Shan–Chen lattice Boltzmann library (declared in
// include/lbm_axi.h): parameter validation, workspace layout, launches of
// the fused step kernel on the caller's stream, moments and FP64
// reductions, state checkpointing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lbm_axi.h"
#include "common.hpp"
#include "lattice.hpp"
#include "step_kernel.hpp"
#include "strip_kernel.hpp"

namespace {

using namespace lbm_host;

// Tile shapes of the fused kernel (chosen by timing on MI355X, with the two
// state buffers alternating as in a run).  Large lattices use 64 x 16 tiles
// of 512 threads, two or more workgroups per compute unit.  In FP64 each XCD
// takes runs of whole tile rows (4096 x 512 on unpadded planes: 82 us per
// step, against 89-94 us for 64 x 32 tiles of 1024 threads in r-fastest
// order; 76 us with the padded planes below).  In FP32 each XCD
// takes a slab of tile columns, and the stores are written through L2 to the
// memory-side cache, which holds both FP32 buffers (35 us, against 40 us
// with row runs and cached stores; neither helps FP64, whose two buffers do
// not fit).  Lattices with fewer than 4 large tiles per compute unit use
// 32 x 16 tiles (512 threads), which keep more compute units busy.
struct Shape {
    int tz, tr;
};
constexpr Shape kShape[2] = {{64, 16}, {32, 16}};  // [0] large, [1] small
constexpr int kNT64 = 512, kNT32 = 512, kNTSmall = 512;

int tiles_of(const lbm_axi_params* p, int c) {
    return ((p->nz + kShape[c].tz - 1) / kShape[c].tz) * ((p->nr + kShape[c].tr - 1) / kShape[c].tr);
}

// Population planes inside the library are padded by kPlanePadBytes (8 KiB):
// planes exactly 2^k bytes apart (16 MiB at 4096 x 512 in FP64) map the same
// node of every plane onto the same memory channels.  The padded pitch made
// the 4096 x 512 step 5% faster in FP64 and 12% in FP32 (8 KiB beat 4 and
// 16 KiB).  The state a caller sees (get/set_state, record) keeps the plain
// [9][nr][nz] layout.
struct Layout {
    size_t state_bytes;   // the caller's view of one state: 9 nz nr values
    long long pitch;      // plane pitch of the library's buffers, in elements
    size_t buf_bytes;     // one population buffer: 9 pitch values
    size_t off_b;         // second buffer
    size_t off_partials;  // [max blocks][4] doubles
    size_t off_red;       // [4] doubles
    size_t off_iface;     // interface scratch: R(z) [nz], rho on row 0 [nz], outputs [8], drops [1 + 2 max]
    size_t off_open;      // inlet velocity profile [2][nz] (open rows)
    size_t off_h;         // H_z, H_r, mass source [3][n] (mid-link source option only)
    size_t total;
    int cfg;              // tile shape in use
    int tiles_z, tiles_r, nblocks;
};

// offsets do not depend on the tile shape (the partials are sized for the
// shape with more tiles), so the workspace size is a function of p alone
Layout layout_of(const lbm_axi_params* p, int cfg) {
    Layout L{};
    const size_t n = (size_t)p->nz * p->nr;
    L.state_bytes = 9 * n * storage_size(p->precision);
    L.pitch = (long long)n + kPlanePadBytes / (long long)storage_size(p->precision);
    L.buf_bytes = 9 * (size_t)L.pitch * storage_size(p->precision);
    L.cfg = cfg;
    L.tiles_z = (p->nz + kShape[cfg].tz - 1) / kShape[cfg].tz;
    L.tiles_r = (p->nr + kShape[cfg].tr - 1) / kShape[cfg].tr;
    L.nblocks = L.tiles_z * L.tiles_r;
    const int max_blocks = tiles_of(p, 1) > tiles_of(p, 0) ? tiles_of(p, 1) : tiles_of(p, 0);
    L.off_b = align_up(L.buf_bytes);
    L.off_partials = L.off_b + align_up(L.buf_bytes);
    L.off_red = L.off_partials + align_up((size_t)max_blocks * 4 * sizeof(double));
    L.off_iface = L.off_red + align_up(4 * sizeof(double));
    L.off_open = L.off_iface + align_up((2 * (size_t)p->nz + 8 + 1 + 2 * LBM_AXI_MAX_DROPS) * sizeof(double));
    L.off_h = L.off_open + align_up(2 * (size_t)p->nz * sizeof(double));
    L.total = L.off_h + ((p->flags & LBM_AXI_FLAG_MIDLINK) ? align_up(3 * n * sizeof(double)) : 0);
    return L;
}

// large tiles when they give at least 4 workgroups per compute unit
int pick_shape(const lbm_axi_params* p) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    return tiles_of(p, 0) >= 4 * cus ? 0 : 1;
}

// fixed-order sum of the per-block partials into out[4]
__global__ void finalize_reduce_kernel(const double* partials, int nblocks, double* out) {
    __shared__ double s[4][256];
    const int t = threadIdx.x;
    for (int m = 0; m < 4; ++m) {
        double v = 0.0;
        for (int b = t; b < nblocks; b += 256) v += partials[(long long)b * 4 + m];
        s[m][t] = v;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int m = 0; m < 4; ++m) s[m][t] += s[m][t + w];
        __syncthreads();
    }
    if (t < 4) out[t] = s[t][0];
}

// One thread per column: the interface radius R(z) (outermost rho_mid
// crossing along r, the rows read from the top down so that the first
// crossing found is the outermost) and rho on the row next to the axis.
template <class P>
__global__ void interface_columns_kernel(const typename P::S* __restrict__ f, long long plane, int nz, int nr,
                                         double rho_ref, double rho_mid, double* __restrict__ radius,
                                         double* __restrict__ rho_axis) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nz) return;
    auto rho_at = [&](int r) {
        const long long x = (long long)r * nz + z;
        double s = 0.0;
        for (int i = 0; i < lbm::kQ; ++i) s += double(f[i * plane + x]);
        return P::kShift ? s + rho_ref : s;
    };
    double R = 0.0, above = 0.0;
    for (int r = nr - 1; r >= 0; --r) {
        const double a = rho_at(r);
        if (a >= rho_mid) {
            R = (r == nr - 1) ? nr - 0.5 : (r + 0.5) + (a - rho_mid) / (a - above);
            break;
        }
        above = a;
    }
    radius[z] = R;
    rho_axis[z] = rho_at(0);
}

// single workgroup: min / max over the columns in a fixed order, then the
// outputs of lbm_axi_interface
template <class P>
__global__ void interface_reduce_kernel(const typename P::S* __restrict__ f, long long plane, int nz, int nr,
                                        double rho_ref, double G, double rho0, int z_col,
                                        const double* __restrict__ radius, const double* __restrict__ rho_axis,
                                        double* __restrict__ out) {
    __shared__ double s_min[256], s_max[256], s_ax[256];
    const int t = threadIdx.x;
    double mn = 1e300, mx = -1e300, ax = 1e300;
    for (int z = t; z < nz; z += 256) {
        mn = fmin(mn, radius[z]);
        mx = fmax(mx, radius[z]);
        ax = fmin(ax, rho_axis[z]);
    }
    s_min[t] = mn;
    s_max[t] = mx;
    s_ax[t] = ax;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (t < k) {
            s_min[t] = fmin(s_min[t], s_min[t + k]);
            s_max[t] = fmax(s_max[t], s_max[t + k]);
            s_ax[t] = fmin(s_ax[t], s_ax[t + k]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const long long top = (long long)(nr - 1) * nz;
        double rout = 0.0;
        for (int i = 0; i < lbm::kQ; ++i) rout += double(f[i * plane + top]);
        if (P::kShift) rout += rho_ref;
        const double rin = rho_axis[z_col];
        auto pressure = [&](double rho) {
            const double psi = rho0 * (1.0 - exp(-rho / rho0));
            return rho / 3.0 + G / 6.0 * psi * psi;
        };
        out[0] = radius[z_col];
        out[1] = s_min[0];
        out[2] = s_max[0];
        out[3] = s_ax[0];
        out[4] = rin;
        out[5] = rout;
        out[6] = pressure(rin) - pressure(rout);
    }
}

// one thread: the drops along the axis (runs of columns whose row 0 is at
// or above rho_mid, periodic in z), listed from the first gas column on;
// volume sum_z pi R(z)^2 and volume-weighted centre of each.  out[0] is the
// count (-1: every axis node is liquid), then max_drops volumes, then
// max_drops centres.
__global__ void drops_scan_kernel(const double* __restrict__ radius, const double* __restrict__ rho_axis, int nz,
                                  double rho_mid, int max_drops, double* __restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int start = -1;
    for (int z = 0; z < nz; ++z) {
        if (rho_axis[z] < rho_mid) {
            start = z;
            break;
        }
    }
    if (start < 0) {
        out[0] = -1.0;
        return;
    }
    auto col = [&](int k) { return start + k < nz ? start + k : start + k - nz; };
    int n = 0, k = 0;
    while (k < nz) {
        if (rho_axis[col(k)] < rho_mid) {
            ++k;
            continue;
        }
        double v = 0.0, m = 0.0;
        while (k < nz && rho_axis[col(k)] >= rho_mid) {
            const double R = radius[col(k)];
            const double w = 3.141592653589793 * (R * R);
            v += w;
            m += w * double(start + k);
            ++k;
        }
        if (n < max_drops) {
            out[1 + n] = v;
            out[1 + max_drops + n] = fmod(m / v, double(nz));
        }
        ++n;
    }
    out[0] = double(n);
}

}  // namespace

struct lbm_axi_ctx {
    lbm_axi_params p;
    int strip_rows = 0;  // chunk height of the row-marching step kernel, 0: tile kernel
    int alternate = 0;   // tile kernel: walk the tiles in reverse order on every other step
    int colmajor = 0;    // tile kernel: each XCD walks its rows of tiles column by column
    int pairs = 0;       // tile kernel: z-adjacent node pairs per thread (large tiles, steps only)
    // two steps (from buffer 0 and from buffer 1) captured as a graph, replayed
    // by lbm_axi_step on small lattices; dropped when the launch arguments change
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    char* ws;
    size_t ws_bytes;
    Layout L;
    int cur;  // index of the buffer holding the current state
    hipStream_t stream;
    int in_row = -1, out_row = -1;  // open rows (lbm_axi_set_open), -1: none
    double rho_in = 1.0, rho_out = 1.0;
};

namespace {

void* state_ptr(lbm_axi_ctx* h, int which) { return h->ws + (which == 0 ? 0 : h->L.off_b); }

lbm::StepArgs make_args(lbm_axi_ctx* h) {
    lbm::StepArgs a{};
    a.plane = h->L.pitch;
    a.state_bytes = (unsigned)h->L.buf_bytes;
    a.nz = h->p.nz;
    a.nr = h->p.nr;
    a.tiles_z = h->L.tiles_z;
    a.big_nz = h->p.nz >= kShape[h->L.cfg].tz + 6 ? 1 : 0;
    a.wall = h->p.wall;
    a.axisym = h->p.axisym;
    a.opts = lbm_host::option_bits(h->p.flags);
    a.G = h->p.G;
    a.tau = h->p.tau;
    a.rho0 = h->p.psi_rho0;
    a.gz = h->p.gz;
    a.rho_ref = h->p.precision == LBM_AXI_FP64 ? 0.0 : h->p.rho_ref;
    a.in_row = h->in_row;
    a.out_row = h->out_row;
    a.rho_bc_in = h->rho_in;
    a.rho_bc_out = h->rho_out;
    a.u_in = reinterpret_cast<const double*>(h->ws + h->L.off_open);
    if (h->in_row >= 0 || h->out_row >= 0) a.opts |= 8;
    a.colmajor = h->colmajor;
    a.h_in = reinterpret_cast<const double*>(h->ws + h->L.off_h);
    return a;
}

template <bool kMoments, int kOpt>
void launch_shape(lbm_axi_ctx* h, const lbm::StepArgs& a) {
    const dim3 grid(h->L.nblocks);
    const bool f64 = h->p.precision == LBM_AXI_FP64;
    if constexpr (!kMoments && kOpt >= 0) {
        if (h->strip_rows > 0) {
            lbm::StripArgs sa;
            sa.chunk_rows = h->strip_rows;
            sa.chunks = (h->p.nr + sa.chunk_rows - 1) / sa.chunk_rows;
            const int bands = (h->p.nz + lbm::kStripW - 1) / lbm::kStripW;
            const dim3 sgrid(bands * sa.chunks);
            if (f64)
                hipLaunchKernelGGL((lbm::axi_strip_kernel<lbm::PrecF64, kOpt, 0>), sgrid, dim3(lbm::kStripNT), 0,
                                   h->stream, a, sa);
            else
                hipLaunchKernelGGL((lbm::axi_strip_kernel<lbm::PrecF32S, kOpt, 16>), sgrid, dim3(lbm::kStripNT), 0,
                                   h->stream, a, sa);
            return;
        }
    }
    if constexpr (!kMoments) {
        if (h->L.cfg == 0 && h->pairs) {
            if (f64)
                hipLaunchKernelGGL((lbm::axi_tile_kernel<lbm::PrecF64, 64, 16, kNT64, false, kOpt, false, 0, true>),
                                   grid, dim3(kNT64), 0, h->stream, a);
            else
                hipLaunchKernelGGL((lbm::axi_tile_kernel<lbm::PrecF32S, 64, 16, kNT32, false, kOpt, true, 16, true>),
                                   grid, dim3(kNT32), 0, h->stream, a);
            return;
        }
    }
    if (h->L.cfg == 0) {
        if (f64)
            hipLaunchKernelGGL((lbm::axi_tile_kernel<lbm::PrecF64, 64, 16, kNT64, kMoments, kOpt>), grid, dim3(kNT64),
                               0, h->stream, a);
        else
            hipLaunchKernelGGL((lbm::axi_tile_kernel<lbm::PrecF32S, 64, 16, kNT32, kMoments, kOpt, true, 16>), grid,
                               dim3(kNT32), 0, h->stream, a);
    } else {
        if (f64)
            hipLaunchKernelGGL((lbm::axi_tile_kernel<lbm::PrecF64, 32, 16, kNTSmall, kMoments, kOpt>), grid,
                               dim3(kNTSmall), 0, h->stream, a);
        else
            hipLaunchKernelGGL((lbm::axi_tile_kernel<lbm::PrecF32S, 32, 16, kNTSmall, kMoments, kOpt>), grid,
                               dim3(kNTSmall), 0, h->stream, a);
    }
}

// the forcing and wall-reading options are compile-time choices of the
// kernel, the boundary options (z walls, open rows) are read at run time;
// the moments do not depend on the forcing option
template <bool kMoments>
int launch_tile(lbm_axi_ctx* h, const lbm::StepArgs& a) {
    const int o = kMoments ? (a.opts & ~1) : a.opts;
    switch (o) {
        case 0: launch_shape<kMoments, 0>(h, a); break;
        case 1: launch_shape<kMoments, 1>(h, a); break;
        case 2: launch_shape<kMoments, 2>(h, a); break;
        case 3: launch_shape<kMoments, 3>(h, a); break;
        default: launch_shape<kMoments, -1>(h, a); break;
    }
    HIP_TRY(hipGetLastError(), "step kernel launch");
    return LBM_AXI_OK;
}

void drop_graphs(lbm_axi_ctx* h) {
    for (auto& g : h->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// one step from state fin into state fout (the handle's layout); with the
// mid-link source, the moments pass that writes H and the mass source first
int step_into(lbm_axi_ctx* h, lbm::StepArgs a, const void* fin, void* fout) {
    a.fin = fin;
    a.fout = fout;
    if (a.opts & 16) {
        lbm::StepArgs m = a;
        m.h_out = reinterpret_cast<double*>(h->ws + h->L.off_h);
        const int rc = launch_tile<true>(h, m);
        if (rc != LBM_AXI_OK) return rc;
    }
    return launch_tile<false>(h, a);
}

}  // namespace

extern "C" {

int lbm_axi_check_params(const lbm_axi_params* p) {
    const int rc = check_params(p);
    if (rc != LBM_AXI_OK) return rc;
    return stability_warning(p->G);
}

size_t lbm_axi_workspace_bytes(const lbm_axi_params* p) {
    if (check_params(p) != LBM_AXI_OK) return 0;
    return layout_of(p, 0).total;
}

int lbm_axi_create(const lbm_axi_params* p, const double* d_rho0, const double* d_uz0, const double* d_ur0,
                   void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_axi_t* out) {
    int rc = check_params(p);
    if (rc != LBM_AXI_OK) return rc;
    if (!out) return fail(LBM_AXI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_rho0) return fail(LBM_AXI_EINVAL, "d_rho0 is NULL");
    if (!d_workspace) return fail(LBM_AXI_EINVAL, "workspace is NULL");
    if ((uintptr_t)d_workspace % kAlign != 0) return fail(LBM_AXI_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = layout_of(p, pick_shape(p));
    if (ws_bytes < L.total)
        return fail(LBM_AXI_ENOMEM, "workspace too small: %zu bytes, need %zu", ws_bytes, L.total);
    auto* h = new (std::nothrow) lbm_axi_ctx{};
    if (!h) return fail(LBM_AXI_ENOMEM, "host allocation failed");
    h->p = *p;
    h->ws = static_cast<char*>(d_workspace);
    h->ws_bytes = ws_bytes;
    h->L = L;
    h->cur = 0;
    h->stream = static_cast<hipStream_t>(hip_stream);
    const long long n = (long long)p->nz * p->nr;
    const int threads = 256;
    const int blocks = (int)((n + threads - 1) / threads);
    const double rho_ref = p->precision == LBM_AXI_FP64 ? 0.0 : p->rho_ref;
    if (p->precision == LBM_AXI_FP64)
        hipLaunchKernelGGL(init_equilibrium_kernel<lbm::PrecF64>, dim3(blocks), dim3(threads), 0, h->stream,
                           static_cast<double*>(state_ptr(h, 0)), d_rho0, d_uz0, d_ur0, n, L.pitch, rho_ref);
    else
        hipLaunchKernelGGL(init_equilibrium_kernel<lbm::PrecF32S>, dim3(blocks), dim3(threads), 0, h->stream,
                           static_cast<float*>(state_ptr(h, 0)), d_rho0, d_uz0, d_ur0, n, L.pitch, rho_ref);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "init kernel launch");
    }
    *out = h;
    return stability_warning(p->G);
}

namespace {
// lattices at most this large replay their steps as graphs (the launch
// overhead is a visible share of a step there: 256 x 128 takes 7.5 us)
constexpr long long kGraphMaxNodes = 1 << 18;

// capture two steps, from buffer `from` and back, on the handle's stream
int ensure_graph(lbm_axi_ctx* h, int from) {
    if (h->graph[from]) return LBM_AXI_OK;
    lbm::StepArgs a = make_args(h);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "graph capture begin");
    int rc = LBM_AXI_OK;
    for (int k = 0; k < 2 && rc == LBM_AXI_OK; ++k) {
        const int c = k == 0 ? from : 1 - from;
        a.reverse = h->alternate ? c : 0;
        rc = step_into(h, a, state_ptr(h, c), state_ptr(h, 1 - c));
    }
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc != LBM_AXI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture end");
    const hipError_t ei = hipGraphInstantiate(&h->graph[from], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the executable graph keeps what it needs
    if (ei != hipSuccess) {
        h->graph[from] = nullptr;
        return hip_fail(ei, "graph instantiate");
    }
    return LBM_AXI_OK;
}
}  // namespace

int lbm_axi_step(lbm_axi_t h, int64_t n) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (n < 0) return fail(LBM_AXI_EINVAL, "n must be >= 0");
    // a stream the caller is capturing into a graph of its own gets the
    // launches themselves; the buffer parity is host state, so a capture
    // that is to be replayed must hold an even number of steps
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (h->stream != nullptr) HIP_TRY(hipStreamIsCapturing(h->stream, &cs), "stream capture status");
    const bool captured = cs != hipStreamCaptureStatusNone;
    if (captured && (n & 1))
        return fail(LBM_AXI_EINVAL, "n must be even while the stream is being captured (got %lld)", (long long)n);
    int64_t done = 0;
    // pairs of steps as graph replays: small lattices, a capturable stream
    // (not the null stream) that nobody captures
    if (n >= 4 && h->stream != nullptr && !captured && (long long)h->p.nz * h->p.nr <= kGraphMaxNodes) {
        const int rc = ensure_graph(h, h->cur);
        if (rc != LBM_AXI_OK) return rc;
        for (; done + 2 <= n; done += 2) HIP_TRY(hipGraphLaunch(h->graph[h->cur], h->stream), "graph launch");
    }
    lbm::StepArgs a = make_args(h);
    for (; done < n; ++done) {
        a.reverse = h->alternate ? h->cur : 0;
        const int rc = step_into(h, a, state_ptr(h, h->cur), state_ptr(h, 1 - h->cur));
        if (rc != LBM_AXI_OK) return rc;
        h->cur = 1 - h->cur;
    }
    return LBM_AXI_OK;
}

int lbm_axi_moments(lbm_axi_t h, double* d_rho, double* d_uz, double* d_ur) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    lbm::StepArgs a = make_args(h);
    a.fin = state_ptr(h, h->cur);
    a.rho_out = d_rho;
    a.uz_out = d_uz;
    a.ur_out = d_ur;
    a.partials = nullptr;
    return launch_tile<true>(h, a);
}

int lbm_axi_reduce(lbm_axi_t h, double* h_out) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (!h_out) return fail(LBM_AXI_EINVAL, "h_out is NULL");
    lbm::StepArgs a = make_args(h);
    a.fin = state_ptr(h, h->cur);
    a.partials = reinterpret_cast<double*>(h->ws + h->L.off_partials);
    int rc = launch_tile<true>(h, a);
    if (rc != LBM_AXI_OK) return rc;
    double* d_red = reinterpret_cast<double*>(h->ws + h->L.off_red);
    hipLaunchKernelGGL(finalize_reduce_kernel, dim3(1), dim3(256), 0, h->stream, a.partials, h->L.nblocks, d_red);
    HIP_TRY(hipGetLastError(), "reduce kernel launch");
    HIP_TRY(hipMemcpyAsync(h_out, d_red, LBM_AXI_NREDUCE * sizeof(double), hipMemcpyDeviceToHost, h->stream),
            "reduce copy");
    HIP_TRY(hipStreamSynchronize(h->stream), "reduce synchronize");
    for (int k = 0; k < LBM_AXI_NREDUCE; ++k)
        if (!std::isfinite(h_out[k])) return fail(LBM_AXI_ENONFINITE, "diagnostic %d is not finite", k);
    return LBM_AXI_OK;
}

int lbm_axi_interface(lbm_axi_t h, double rho_mid, int32_t z_col, double* d_radius, double* h_out) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (!h_out) return fail(LBM_AXI_EINVAL, "h_out is NULL");
    if (z_col < 0 || z_col >= h->p.nz) return fail(LBM_AXI_EINVAL, "z_col out of range (0 .. %d)", h->p.nz - 1);
    if (!std::isfinite(rho_mid)) return fail(LBM_AXI_EINVAL, "rho_mid must be finite");
    double* scratch = reinterpret_cast<double*>(h->ws + h->L.off_iface);
    double* radius = d_radius ? d_radius : scratch;
    double* rho_axis = scratch + h->p.nz;
    double* d_out = scratch + 2 * (size_t)h->p.nz;
    const long long plane = h->L.pitch;
    const double rho_ref = h->p.precision == LBM_AXI_FP64 ? 0.0 : h->p.rho_ref;
    const dim3 cols((h->p.nz + 255) / 256);
    if (h->p.precision == LBM_AXI_FP64) {
        const double* f = static_cast<const double*>(state_ptr(h, h->cur));
        hipLaunchKernelGGL(interface_columns_kernel<lbm::PrecF64>, cols, dim3(256), 0, h->stream, f, plane, h->p.nz,
                           h->p.nr, rho_ref, rho_mid, radius, rho_axis);
        hipLaunchKernelGGL(interface_reduce_kernel<lbm::PrecF64>, dim3(1), dim3(256), 0, h->stream, f, plane,
                           h->p.nz, h->p.nr, rho_ref, h->p.G, h->p.psi_rho0, z_col, radius, rho_axis, d_out);
    } else {
        const float* f = static_cast<const float*>(state_ptr(h, h->cur));
        hipLaunchKernelGGL(interface_columns_kernel<lbm::PrecF32S>, cols, dim3(256), 0, h->stream, f, plane, h->p.nz,
                           h->p.nr, rho_ref, rho_mid, radius, rho_axis);
        hipLaunchKernelGGL(interface_reduce_kernel<lbm::PrecF32S>, dim3(1), dim3(256), 0, h->stream, f, plane,
                           h->p.nz, h->p.nr, rho_ref, h->p.G, h->p.psi_rho0, z_col, radius, rho_axis, d_out);
    }
    HIP_TRY(hipGetLastError(), "interface kernel launch");
    HIP_TRY(hipMemcpyAsync(h_out, d_out, LBM_AXI_NINTERFACE * sizeof(double), hipMemcpyDeviceToHost, h->stream),
            "interface copy");
    HIP_TRY(hipStreamSynchronize(h->stream), "interface synchronize");
    return LBM_AXI_OK;
}

int lbm_axi_set_open(lbm_axi_t h, int32_t in_row, double rho_in, const double* d_uz_in, const double* d_ur_in,
                     int32_t out_row, double rho_out) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    const int nr = h->p.nr;
    if (in_row < -1 || in_row >= nr) return fail(LBM_AXI_EINVAL, "in_row out of range (-1 .. %d)", nr - 1);
    if (out_row < -1 || out_row >= nr) return fail(LBM_AXI_EINVAL, "out_row out of range (-1 .. %d)", nr - 1);
    if (out_row == 0) return fail(LBM_AXI_EINVAL, "out_row must be >= 1 (it takes the velocity of the row below)");
    if (in_row >= 0 && out_row >= 0 && out_row <= in_row) return fail(LBM_AXI_EINVAL, "out_row must lie above in_row");
    if (in_row >= 0 && (!d_uz_in || !d_ur_in)) return fail(LBM_AXI_EINVAL, "inlet velocity profile is NULL");
    if ((in_row >= 0 || out_row >= 0) && (h->p.flags & LBM_AXI_FLAG_MIDLINK))
        return fail(LBM_AXI_EUNSUP, "open rows do not combine with LBM_AXI_FLAG_MIDLINK");
    if (in_row >= 0 && !(rho_in > 0.0 && std::isfinite(rho_in))) return fail(LBM_AXI_EINVAL, "rho_in must be > 0");
    if (out_row >= 0 && !(rho_out > 0.0 && std::isfinite(rho_out))) return fail(LBM_AXI_EINVAL, "rho_out must be > 0");
    if (in_row >= 0) {
        double* prof = reinterpret_cast<double*>(h->ws + h->L.off_open);
        const size_t bytes = (size_t)h->p.nz * sizeof(double);
        HIP_TRY(hipMemcpyAsync(prof, d_uz_in, bytes, hipMemcpyDeviceToDevice, h->stream), "inlet profile copy");
        HIP_TRY(hipMemcpyAsync(prof + h->p.nz, d_ur_in, bytes, hipMemcpyDeviceToDevice, h->stream),
                "inlet profile copy");
    }
    h->in_row = in_row;
    h->out_row = out_row;
    if (in_row >= 0 || out_row >= 0) h->strip_rows = 0;  // open rows run on the tile kernel
    drop_graphs(h);
    h->rho_in = rho_in;
    h->rho_out = rho_out;
    return LBM_AXI_OK;
}

int lbm_axi_drops(lbm_axi_t h, double rho_mid, int32_t max_drops, int32_t* h_count, double* h_volume,
                  double* h_centre) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (!h_count) return fail(LBM_AXI_EINVAL, "h_count is NULL");
    if (max_drops < 0 || max_drops > LBM_AXI_MAX_DROPS)
        return fail(LBM_AXI_EINVAL, "max_drops out of range (0 .. %d)", LBM_AXI_MAX_DROPS);
    if (max_drops > 0 && (!h_volume || !h_centre)) return fail(LBM_AXI_EINVAL, "h_volume or h_centre is NULL");
    if (!std::isfinite(rho_mid)) return fail(LBM_AXI_EINVAL, "rho_mid must be finite");
    double* scratch = reinterpret_cast<double*>(h->ws + h->L.off_iface);
    double* radius = scratch;
    double* rho_axis = scratch + h->p.nz;
    double* d_out = scratch + 2 * (size_t)h->p.nz + 8;
    const long long plane = h->L.pitch;
    const double rho_ref = h->p.precision == LBM_AXI_FP64 ? 0.0 : h->p.rho_ref;
    const dim3 cols((h->p.nz + 255) / 256);
    if (h->p.precision == LBM_AXI_FP64) {
        const double* f = static_cast<const double*>(state_ptr(h, h->cur));
        hipLaunchKernelGGL(interface_columns_kernel<lbm::PrecF64>, cols, dim3(256), 0, h->stream, f, plane, h->p.nz,
                           h->p.nr, rho_ref, rho_mid, radius, rho_axis);
    } else {
        const float* f = static_cast<const float*>(state_ptr(h, h->cur));
        hipLaunchKernelGGL(interface_columns_kernel<lbm::PrecF32S>, cols, dim3(256), 0, h->stream, f, plane, h->p.nz,
                           h->p.nr, rho_ref, rho_mid, radius, rho_axis);
    }
    hipLaunchKernelGGL(drops_scan_kernel, dim3(1), dim3(64), 0, h->stream, radius, rho_axis, h->p.nz, rho_mid,
                       max_drops, d_out);
    HIP_TRY(hipGetLastError(), "drops kernel launch");
    double host[1 + 2 * LBM_AXI_MAX_DROPS];
    HIP_TRY(hipMemcpyAsync(host, d_out, (1 + 2 * (size_t)max_drops) * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream),
            "drops copy");
    HIP_TRY(hipStreamSynchronize(h->stream), "drops synchronize");
    const int n = (int)host[0];
    *h_count = n;
    for (int k = 0; k < n && k < max_drops; ++k) {
        h_volume[k] = host[1 + k];
        h_centre[k] = host[1 + max_drops + k];
    }
    return LBM_AXI_OK;
}

int lbm_axi_populations(lbm_axi_t h, double* d_f) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (!d_f) return fail(LBM_AXI_EINVAL, "d_f is NULL");
    const long long n = (long long)h->p.nz * h->p.nr;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (h->p.precision == LBM_AXI_FP64)
        hipLaunchKernelGGL(decode_populations_kernel<lbm::PrecF64>, grid, dim3(256), 0, h->stream,
                           static_cast<const double*>(state_ptr(h, h->cur)), h->L.pitch, n, 0.0, d_f);
    else
        hipLaunchKernelGGL(decode_populations_kernel<lbm::PrecF32S>, grid, dim3(256), 0, h->stream,
                           static_cast<const float*>(state_ptr(h, h->cur)), h->L.pitch, n, h->p.rho_ref, d_f);
    HIP_TRY(hipGetLastError(), "populations kernel launch");
    return LBM_AXI_OK;
}

size_t lbm_axi_state_bytes(lbm_axi_t h) { return h ? h->L.state_bytes : 0; }

namespace {
// the nine planes between the library's padded buffers and the caller's
// plain [9][nr][nz] layout
hipError_t copy_planes(lbm_axi_ctx* h, void* dst, bool dst_padded, const void* src, bool src_padded) {
    const size_t row = h->L.state_bytes / 9, padded = h->L.buf_bytes / 9;
    return hipMemcpy2DAsync(dst, dst_padded ? padded : row, src, src_padded ? padded : row, row, 9,
                            hipMemcpyDeviceToDevice, h->stream);
}
}  // namespace

int lbm_axi_get_state(lbm_axi_t h, void* d_dst) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (!d_dst) return fail(LBM_AXI_EINVAL, "d_dst is NULL");
    HIP_TRY(copy_planes(h, d_dst, false, state_ptr(h, h->cur), true), "get_state copy");
    return LBM_AXI_OK;
}

int lbm_axi_set_state(lbm_axi_t h, const void* d_src) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (!d_src) return fail(LBM_AXI_EINVAL, "d_src is NULL");
    HIP_TRY(copy_planes(h, state_ptr(h, h->cur), true, d_src, false), "set_state copy");
    return LBM_AXI_OK;
}

int lbm_axi_record(lbm_axi_t h, int64_t n, void* d_states) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (!d_states) return fail(LBM_AXI_EINVAL, "d_states is NULL");
    if (n < 1) return fail(LBM_AXI_EINVAL, "n must be >= 1");
    // the steps write straight into the record, in the caller's plain
    // layout: one copy in, one copy back
    char* dst = static_cast<char*>(d_states);
    const size_t sb = h->L.state_bytes;
    HIP_TRY(copy_planes(h, dst, false, state_ptr(h, h->cur), true), "record copy");
    lbm::StepArgs a = make_args(h);
    a.plane = (long long)h->p.nz * h->p.nr;
    a.state_bytes = (unsigned)sb;
    for (int64_t j = 1; j < n; ++j) {
        const int rc = step_into(h, a, dst + (size_t)(j - 1) * sb, dst + (size_t)j * sb);
        if (rc != LBM_AXI_OK) return rc;
    }
    if (n > 1) HIP_TRY(copy_planes(h, state_ptr(h, h->cur), true, dst + (size_t)(n - 1) * sb, false), "record copy");
    return LBM_AXI_OK;
}

int lbm_axi_set_kernel(lbm_axi_t h, int32_t kind, int32_t chunk_rows) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    if (kind == LBM_AXI_KERNEL_TILE || kind == LBM_AXI_KERNEL_TILE_ALTERNATE || kind == LBM_AXI_KERNEL_TILE_COLUMNS ||
        kind == LBM_AXI_KERNEL_TILE_PAIRS) {
        h->strip_rows = 0;
        h->alternate = kind == LBM_AXI_KERNEL_TILE_ALTERNATE;
        h->colmajor = kind == LBM_AXI_KERNEL_TILE_COLUMNS;
        h->pairs = kind == LBM_AXI_KERNEL_TILE_PAIRS;
        drop_graphs(h);
        return LBM_AXI_OK;
    }
    if (kind != LBM_AXI_KERNEL_STRIP)
        return fail(LBM_AXI_EINVAL,
                    "kind must be LBM_AXI_KERNEL_TILE, _STRIP, _TILE_ALTERNATE, _TILE_COLUMNS or _TILE_PAIRS");
    if (chunk_rows < 1) return fail(LBM_AXI_EINVAL, "chunk_rows must be >= 1 (got %d)", chunk_rows);
    if (h->p.nz < lbm::kStripW + 6)
        return fail(LBM_AXI_EUNSUP, "the row-marching kernel needs nz >= %d (got %d)", lbm::kStripW + 6, h->p.nz);
    if ((option_bits(h->p.flags) & ~3) != 0 || h->in_row >= 0 || h->out_row >= 0)
        return fail(LBM_AXI_EUNSUP, "the row-marching kernel supports the Guo and wall-derivative options only");
    h->strip_rows = chunk_rows;
    drop_graphs(h);
    return LBM_AXI_OK;
}

int lbm_axi_set_stream(lbm_axi_t h, void* hip_stream) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    h->stream = static_cast<hipStream_t>(hip_stream);
    return LBM_AXI_OK;
}

int lbm_axi_set_coupling(lbm_axi_t h, double G, double tau) {
    if (!h) return fail(LBM_AXI_EINVAL, "handle is NULL");
    lbm_axi_params q = h->p;
    q.G = G;
    q.tau = tau;
    int rc = check_params(&q);
    if (rc != LBM_AXI_OK) return rc;
    h->p = q;
    drop_graphs(h);
    return stability_warning(G);
}

void lbm_axi_destroy(lbm_axi_t h) {
    if (!h) return;
    drop_graphs(h);
    delete h;
}

const char* lbm_axi_last_error(void) { return lbm_host::g_last_error.c_str(); }

}  // extern "C"
