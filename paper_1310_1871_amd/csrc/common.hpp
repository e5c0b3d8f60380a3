// Host-side helpers shared by the library's C ABI translation units:
// thread-local error message, parameter validation, the initial-equilibrium
// kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/lbm_axi.h"
#include "lattice.hpp"
#include "step_kernel.hpp"

namespace lbm_host {

inline thread_local std::string g_last_error;

inline int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

inline int hip_fail(hipError_t e, const char* what) {
    return fail(LBM_AXI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline size_t storage_size(int precision) { return precision == LBM_AXI_FP64 ? sizeof(double) : sizeof(float); }

// padding, in bytes, of each population plane in the library's own
// buffers (single lattices and batch instances): planes exactly 2^k bytes
// apart put the same node of every plane on the same memory channels
constexpr long long kPlanePadBytes = 8192;

inline int check_params(const lbm_axi_params* p) {
    if (!p) return fail(LBM_AXI_EINVAL, "params is NULL");
    if (p->nz < 1) return fail(LBM_AXI_EINVAL, "nz must be >= 1 (got %d)", p->nz);
    if (p->nr < 6) return fail(LBM_AXI_EINVAL, "nr must be >= 6 for the derivative stencils (got %d)", p->nr);
    // (with room for the padding of the buffers' planes)
    if (9.0 * ((double)p->nz * (double)p->nr * (p->precision == LBM_AXI_FP64 ? 8.0 : 4.0) + (double)kPlanePadBytes) >=
        4294967296.0)
        return fail(LBM_AXI_EINVAL, "grid too large: the population state must stay below 4 GiB");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_AXI_EINVAL, "tau must be > 1/2 (got %g)", p->tau);
    if (!std::isfinite(p->G)) return fail(LBM_AXI_EINVAL, "G must be finite");
    if (!(p->psi_rho0 > 0.0) || !std::isfinite(p->psi_rho0)) return fail(LBM_AXI_EINVAL, "psi_rho0 must be > 0");
    if (!std::isfinite(p->gz)) return fail(LBM_AXI_EINVAL, "gz must be finite");
    if (p->wall != LBM_AXI_WALL_NOSLIP && p->wall != LBM_AXI_WALL_FREESLIP)
        return fail(LBM_AXI_EINVAL, "wall must be 0 (no-slip) or 1 (free-slip)");
    if (p->axisym != 0 && p->axisym != 1) return fail(LBM_AXI_EINVAL, "axisym must be 0 or 1");
    if (p->precision != LBM_AXI_FP64 && p->precision != LBM_AXI_FP32_SHIFTED)
        return fail(LBM_AXI_EINVAL, "precision must be 0 (FP64) or 1 (FP32 shifted)");
    if ((p->flags & ~(LBM_AXI_FLAG_GUO | LBM_AXI_FLAG_NO_WALL_DERIV | LBM_AXI_FLAG_ZWALLS | LBM_AXI_FLAG_MIDLINK)) !=
        0)
        return fail(LBM_AXI_EUNSUP,
                    "flags may combine LBM_AXI_FLAG_GUO, LBM_AXI_FLAG_NO_WALL_DERIV, LBM_AXI_FLAG_ZWALLS and "
                    "LBM_AXI_FLAG_MIDLINK only (got %d)",
                    p->flags);
    if ((p->flags & LBM_AXI_FLAG_MIDLINK) && (p->flags & LBM_AXI_FLAG_ZWALLS))
        return fail(LBM_AXI_EUNSUP, "LBM_AXI_FLAG_MIDLINK does not combine with LBM_AXI_FLAG_ZWALLS");
    if ((p->flags & LBM_AXI_FLAG_ZWALLS) && p->nz < 8)
        return fail(LBM_AXI_EINVAL, "nz must be >= 8 with LBM_AXI_FLAG_ZWALLS (got %d)", p->nz);
    if (!std::isfinite(p->rho_ref)) return fail(LBM_AXI_EINVAL, "rho_ref must be finite");
    return LBM_AXI_OK;
}

// Sec. II.D: as a rule of thumb the scheme stays stable up to a density
// ratio of about 35, reached at G = -6; stronger coupling is accepted with a
// warning.  Returns LBM_AXI_WARN_STABILITY (message set) or LBM_AXI_OK.
inline int stability_warning(double G) {
    if (G < -6.0)
        return fail(LBM_AXI_WARN_STABILITY,
                    "G = %g < -6: beyond the stability rule of thumb (density ratio <= 35 for G >= -6)", G);
    return LBM_AXI_OK;
}

// kernel option bits of a validated flags field (1 Guo forcing, 2 no
// derivative terms across the wall, 4 z walls, 16 mid-link source; 8, open
// rows, is set by lbm_axi_set_open)
inline int option_bits(int flags) {
    return ((flags & LBM_AXI_FLAG_GUO) ? 1 : 0) | ((flags & LBM_AXI_FLAG_NO_WALL_DERIV) ? 2 : 0) |
           ((flags & LBM_AXI_FLAG_ZWALLS) ? 4 : 0) | ((flags & LBM_AXI_FLAG_MIDLINK) ? 16 : 0);
}

// f_i = f^eq_i(rho, u) with u^eq = u (initial state, no force shift)
template <class P>
__global__ void init_equilibrium_kernel(typename P::S* f, const double* rho, const double* uz,
                                        const double* ur, long long n, long long pitch, double rho_ref) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const double r = rho[x];
    const double vz = uz ? uz[x] : 0.0;
    const double vr = ur ? ur[x] : 0.0;
    const double qq = 1.5 * (vz * vz + vr * vr);
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) {
        const double cu = lbm::cz(i) * vz + lbm::cr(i) * vr;
        const double poly = 3.0 * cu + 4.5 * cu * cu - qq;
        const double w = lbm::weight(i);
        double v = P::kShift ? w * ((r - rho_ref) + r * poly) : w * r * (1.0 + poly);
        f[(long long)i * pitch + x] = typename P::S(v);
    }
}

// the stored populations as FP64 f_i (FP32 shifted storage: + W_i rho_ref,
// in double), from the library's padded layout into [9][n]
template <class P>
__global__ void decode_populations_kernel(const typename P::S* __restrict__ f, long long pitch, long long n,
                                          double rho_ref, double* __restrict__ out) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) {
        const double v = double(f[(long long)i * pitch + x]);
        out[(long long)i * n + x] = P::kShift ? v + lbm::weight(i) * rho_ref : v;
    }
}

}  // namespace lbm_host
