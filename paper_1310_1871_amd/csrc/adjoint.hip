// Hand-written adjoint (vector-Jacobian product) of one time step of the
// axisymmetric Shan–Chen scheme, FP64.
//
// Forward step (Sec. II): f* = C(f; G, tau), f_next = S(f*), with C the
// collision with all its force and source terms and S the push streaming
// with the boundary rules of Sec. II.E.  Given lam_next = dL/df_next the
// kernels below produce lam = (df_next/df)^T lam_next and accumulate
// dL/dG and dL/dtau.
//
// The reverse step is two tile kernels.  In the forward data flow, psi
// feeds the force through the Shan–Chen neighbour sum and the derivative
// stencils (reach 1, 4 and 2 + 2), the force feeds the velocity, and the
// velocity feeds the source through its own stencils (reach 2).  Reversed:
//
//   A (adj_tile_a), one workgroup per tile, one thread per tile node:
//     1. loads f on the tile and a 6-node ring and recomputes rho, j, psi,
//        d_r psi, the 1D d_r psi, the force and the velocity on the tile and
//        a 2-node ring, as the forward kernel does;
//     2. gathers nu = S^T lam_next on the tile and the 2-node ring (the
//        adjoints of the velocity stencils at a node depend only on nu and
//        rho there), and keeps those adjoints in LDS;
//     3. reverses collision, equilibrium and source at each tile node, folds
//        the velocity-stencil adjoints of its neighbours onto it (with the
//        mirror images at the axis and the wall), then reverses the velocity
//        and the force;
//     4. writes lam_p = f-bar + rho-bar + c . j-bar with every term of
//        rho-bar except the part that passes through the psi stencils of
//        other nodes, and for kernel B P = -G psi F-bar (two components) and
//        E = exp(-rho / rho0);
//   B (adj_tile_b): transposes the psi stencils from P (their adjoints are
//     P / (18 r) and -P_r / (18 r^2)), folds the ghost rows onto the rows
//     they mirror, and gives rho-bar_B = psi-bar_B E.
// lam = lam_p + rho-bar_B in every direction.  A single step adds the two in
// place (B's last form); a run keeps lam in the split form between steps
// and the next step's kernel A adds rho-bar_B in its gathers.
//
// Each workgroup sums its nodes' dL/dG and dL/dtau terms in a fixed order
// into its own slot; no atomics, so results are deterministic.
#include <hip/hip_runtime.h>

#include <climits>

#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbm_axi.h"
#include "../../include/lbm_axi_adjoint.h"
#include "common.hpp"
#include "lattice.hpp"

// Scratch of the allocation-free reverse step (lbm_axi_adjoint_step_noalloc):
// a file-scope device array, one per GPU the library runs on, held until the
// process ends.  Host code reaches it only through the address
// hipGetSymbolAddress gives on each device (the array's name is a host-side
// stand-in there).
static __device__ __align__(256) double scratch[LBM_AXI_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

struct TileArgs {
    int nz, nr;
    long long n;  // nz * nr
    double G, tau, rho0, gz;
    int wall;
    int tiles_z;               // tiles along z (tile id = row of tiles * tiles_z + column)
    const double* f;           // [9][n] state f^t
    const double* lam_p;       // [9][n] lam^{t+1}, less rho-bar_B
    const double* rhob_in;     // [n] rho-bar_B of lam^{t+1}; NULL: lam_p is all of lam^{t+1}
    double* lam_out;           // [9][n] A: lam_p of lam^t; final B: lam^t (lam_p plus rho-bar_B, in place)
    double* pz;                // [n] P_z = -G psi F-bar_z
    double* pr;                // [n] P_r = -G psi F-bar_r
    double* ex;                // [n] E = exp(-rho / rho0)
    double* rhob_out;          // [n] B: rho-bar_B of lam^t
    // the small-lattice kernel A: P and E of the previous reverse step (that
    // of lam^{t+1}), from which it forms rho-bar_B of lam^{t+1} itself; NULL:
    // lam_p is all of lam^{t+1}
    const double* pz_in;
    const double* pr_in;
    const double* ex_in;
    double* part;              // [tiles][2] dL/dG, dL/dtau of each tile
    int accumulate;            // 1: add to part (the running sums of a run), 0: overwrite
};

// tile geometry: TZ x TR nodes, NTH threads (at least one per node: on small
// lattices, where a kernel's time is the length of one workgroup's chain of
// loads, spare threads share the window's loads); window offsets are
// relative to the tile's first node
template <int TZ, int TR, int NTH = TZ * TR>
struct Tile {
    static constexpr int NT = NTH, NTILE = TZ * TR;
    static constexpr int PW = TZ + 12, PH = TR + 12;  // psi: columns and rows [-6, T + 6)
    static constexpr int DW = TZ + 8, DH = TR + 8;    // isotropic d_r psi: [-4, T + 4)
    static constexpr int EW = TZ + 8, EH = TR + 4;    // 1D d_r psi: columns [-4, TZ + 4), rows [-2, TR + 2)
    static constexpr int UW = TZ + 4, UH = TR + 4;    // u and the velocity-stencil adjoints: [-2, T + 2)
    static constexpr int R2N = 4 * (TZ + 4) + 4 * TR;          // ring nodes within 2 of the tile
    static constexpr int OUTN = 8 * (TZ + 12) + 8 * (TR + 4);  // ring nodes 3 to 6 away
    static constexpr int RS = (R2N + OUTN + NT - 1) / NT;      // ring slots per thread
    static_assert(R2N <= NT, "the first ring slot holds every ring node within 2 of the tile");
    static_assert(NT % 64 == 0 && NTILE % 64 == 0 && NT >= NTILE, "whole waves, a thread per tile node");
};

// ring node k of the window: first the nodes within 2 of the tile (rows
// -2, -1, then TR, TR + 1, then columns -2, -1, TZ, TZ + 1 of the tile
// rows), then the nodes 3 to 6 away
template <int TZ, int TR>
__device__ __forceinline__ void ring_pos(int k, int& c, int& y) {
    constexpr int W2 = TZ + 4, W6 = TZ + 12, R2N = 4 * W2 + 4 * TR;
    if (k < 2 * W2) {
        y = -2 + k / W2;
        c = -2 + k % W2;
    } else if (k < 4 * W2) {
        const int j = k - 2 * W2;
        y = TR + j / W2;
        c = -2 + j % W2;
    } else if (k < R2N) {
        const int j = k - 4 * W2, q = j & 3;
        y = j >> 2;
        c = q < 2 ? q - 2 : TZ + q - 2;
    } else {
        const int j = k - R2N;
        if (j < 4 * W6) {
            y = -6 + j / W6;
            c = -6 + j % W6;
        } else if (j < 8 * W6) {
            const int i = j - 4 * W6;
            y = TR + 2 + i / W6;
            c = -6 + i % W6;
        } else {
            const int i = j - 8 * W6, q = i & 7;
            y = -2 + (i >> 3);
            c = q < 4 ? q - 6 : TZ + 2 + (q - 4);
        }
    }
}

// periodic column (any offset)
__device__ __forceinline__ int wrap_col(int z, int nz) {
    z %= nz;
    return z < 0 ? z + nz : z;
}

// the row whose populations a window row reads: rows below the axis and
// beyond the wall take their mirror row (psi is even at both); rows further
// out than one mirror occur only on the last tile of a short lattice, are
// never read by a tile node, and are clamped into the lattice
__device__ __forceinline__ int mirror_even(int y, int nr) {
    if (y < 0) y = -1 - y;
    if (y >= nr) y = 2 * nr - 1 - y;
    return y < 0 ? 0 : (y >= nr ? nr - 1 : y);
}

// tiles in runs of whole tile rows per XCD (workgroup b runs on XCD b mod 8)
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7, x = b & 7, k = b >> 3;
    return x * q + (x < rem ? x : rem) + k;
}

// the same runs walked in blocks 8 tile columns wide spanning the XCD's
// rows, when each run is whole tile rows and a row is a multiple of 8 tiles:
// the workgroups resident on an XCD at one time (two per CU) then cover a
// compact block, whose 6-node rings overlap in the XCD's L2, rather than a
// whole row of tiles, whose windows do not fit it
__device__ __forceinline__ int block_tile(int b, int nb, int tiles_z) {
    const int q = nb >> 3, rem = nb & 7;
    if (rem != 0 || q % tiles_z != 0 || (tiles_z & 7) != 0) return xcd_tile(b, nb);
    const int x = b & 7, k = b >> 3, rows = q / tiles_z;
    const int blk = k / (8 * rows), w = k % (8 * rows);
    return x * q + (w >> 3) * tiles_z + blk * 8 + (w & 7);
}

// Buffer-resource loads and stores: 32-bit byte offsets (one VGPR per
// address instead of a 64-bit pointer pair), the plane of a state or adjoint
// in the scalar offset.  Every buffer here is below 4 GiB (the adjoint takes
// at most 2^32 / 72 nodes); the hardware returns 0 for a load past the
// buffer's end.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc rsrc_of(const void* base, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)(unsigned)bytes, 0x00020000);
}
__device__ __forceinline__ double ld(Rsrc r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void st(Rsrc r, unsigned voff, unsigned soff, double v) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
}

// the push target of direction i from real node (z, r) under the boundary
// rules of Sec. II.E (specular axis; no-slip bounce-back or free-slip
// specular wall): its node index, and in d the direction it arrives in
__device__ __forceinline__ int push_target(int i, int z, int r, int nz, int nr, int wall, int& d) {
    const int ty = r + lbm::cr(i);
    const bool below = ty < 0, above = ty >= nr, back = above && wall == 0;
    int tz = back ? z : z + lbm::cz(i);
    tz = tz < 0 ? tz + nz : (tz >= nz ? tz - nz : tz);
    const int tr = below ? 0 : (above ? (wall == 0 ? r : nr - 1) : ty);
    d = below ? lbm::mirror_r(i) : (above ? (wall == 0 ? lbm::opposite(i) : lbm::mirror_r(i)) : i);
    return tr * nz + tz;
}

// the same target as an offset (dc, dr) from the source node (z, r)
__device__ __forceinline__ void push_offset(int i, int r, int nr, int wall, int& dc, int& dr) {
    const int ty = r + lbm::cr(i);
    const bool below = ty < 0, above = ty >= nr;
    dc = (above && wall == 0) ? 0 : lbm::cz(i);
    dr = below ? -r : (above ? (wall == 0 ? 0 : nr - 1 - r) : lbm::cr(i));
}

// the buffers kernel A reads and writes
struct Bufs {
    Rsrc f, lam, rhob, out, pz, pr, ex;
    unsigned plane;  // bytes of one population plane
};
__device__ __forceinline__ Bufs bufs_of(const TileArgs& a) {
    const size_t nb = (size_t)a.n * sizeof(double);
    Bufs b;
    b.f = rsrc_of(a.f, 9 * nb);
    b.lam = rsrc_of(a.lam_p, 9 * nb);
    b.rhob = rsrc_of(a.rhob_in, a.rhob_in ? nb : 0);
    b.out = rsrc_of(a.lam_out, 9 * nb);
    b.pz = rsrc_of(a.pz, nb);
    b.pr = rsrc_of(a.pr, nb);
    b.ex = rsrc_of(a.ex, nb);
    b.plane = (unsigned)nb;
    return b;
}

// nu_i = lam^{t+1}_d at the push target of direction i
__device__ __forceinline__ double gather_nu(const TileArgs& a, const Bufs& b, int i, int z, int r) {
    int d;
    const unsigned x = (unsigned)push_target(i, z, r, a.nz, a.nr, a.wall, d);
    // without rho-bar_B (rhob_in NULL) its resource has no records and the
    // load reads 0: no branch, which would make each gather wait for the last
    return ld(b.lam, (unsigned)d * b.plane + 8u * x, 0u) + ld(b.rhob, 8u * x, 0u);
}

// the stencils' divisors as factors (a division by a constant that is not
// a power of two is a full IEEE division sequence)
constexpr double kI36 = 1.0 / 36.0, kI12 = 1.0 / 12.0, kI18 = 1.0 / 18.0;

// x y rounded on its own, never contracted into an addition that uses it
__device__ __forceinline__ double mul_rounded(double x, double y) {
#pragma clang fp contract(off)
    return x * y;
}

// ---- psi-bar through the psi stencils of other nodes --------------------
//
// On a region of RZ x RH nodes whose first node is (z0, r0) (z0 may be
// negative, z being periodic; r0 may be negative, rows off the lattice hold
// nothing), from P = -G psi F-bar on the region and a ring around it:
// psi-bar_B, the sum of the transposed SC neighbour sum, the transposed
// d_rr = d_r of d_r psi with the direct d_r psi of F^sym_r, and the
// transposed d_zr (1D d_z of the 1D d_r psi), folded from the ghost rows
// onto the rows they mirror.  Kernel B evaluates it on its tile; kernel A
// of the small-lattice path on its tile and a 3-node ring, for the next
// step's gathers.  Both use these functions, so their values agree bit for
// bit.
template <int RZ, int RH>
struct PsiBar {
    static constexpr int QW = RZ + 8, QH = RH + 16;  // P: columns [-4, RZ + 4), rows [-8, RH + 8)
    static constexpr int GW = RZ + 4, GH = RH + 12;  // adjoint of d_r psi: columns [-2, RZ + 2), rows [-6, RH + 6)
    static constexpr int HH = RH + 12;               // adjoint of the 1D d_r psi: the region's columns, rows [-6, RH + 6)
    double pz[QH][QW], pr[QH][QW];
    double qr[QH][QW];  // d_rr-bar = P_r / (18 r), 0 off the lattice
    double g[GH][GW];
    double h[HH][RZ];
};

// step 1 (every thread): P on the window into LDS.  A thread issues all its
// loads before it uses any (rows off the lattice read past the buffer's
// end, which gives 0, and are zeroed again).
template <int RZ, int RH, int NT, bool kAxi>
__device__ __forceinline__ void psibar_load(PsiBar<RZ, RH>& sb, const double* pz, const double* pr, size_t nb, int z0,
                                            int r0, int nz, int nr, int t) {
    using S = PsiBar<RZ, RH>;
    const Rsrc rpz = rsrc_of(pz, nb), rpr = rsrc_of(pr, nb);
    constexpr int KQ = (S::QH * S::QW + NT - 1) / NT;
    double vz[KQ], vr[KQ];
#pragma unroll
    for (int j = 0; j < KQ; ++j) {
        const int k = t + j * NT, y = k / S::QW - 8, c = k % S::QW - 4;
        const unsigned x = 8u * (unsigned)((r0 + y) * nz + wrap_col(z0 + c, nz));
        vz[j] = ld(rpz, x, 0u);
        vr[j] = ld(rpr, x, 0u);
    }
#pragma unroll
    for (int j = 0; j < KQ; ++j) {
        const int k = t + j * NT, y = k / S::QW - 8, c = k % S::QW - 4;
        if (k < S::QH * S::QW) {
            const bool re = r0 + y >= 0 && r0 + y < nr;
            const double p = re ? vr[j] : 0.0;
            sb.pz[y + 8][c + 4] = re ? vz[j] : 0.0;
            sb.pr[y + 8][c + 4] = p;
            if (kAxi) sb.qr[y + 8][c + 4] = p * kI18 * (1.0 / (r0 + y + 0.5));
        }
    }
}

// step 2 (every thread, after a barrier; axisymmetric terms only): the
// adjoint of d_r psi on the extended rows -2 .. nr + 1 that d_rr reads (the
// transposed isotropic stencil of d_rr-bar, plus the direct use of d_r psi
// on a real row, d_r-bar = -P_r / (18 r^2)), and the adjoint of the 1D d_r
// psi on real rows (the transposed z difference of d_zr-bar = P_z / (18 r))
template <int RZ, int RH, int NT>
__device__ __forceinline__ void psibar_stencils(PsiBar<RZ, RH>& sb, int r0, int nr, int t) {
    using S = PsiBar<RZ, RH>;
    for (int k = t; k < S::GH * S::GW; k += NT) {
        const int y = k / S::GW - 6, c = k % S::GW - 2, yy = r0 + y;
        double v = 0.0;
        if (yy >= -2 && yy < nr + 2) {
            double s = 0.0;
#pragma unroll
            for (int i = 1; i < lbm::kQ; ++i) {
                const int cr = lbm::cr(i), cz = lbm::cz(i);
                if (cr == 0) continue;
                s += 8.0 * cr * sb.qr[y - cr + 8][c - cz + 4];
                s -= cr * sb.qr[y - 2 * cr + 8][c - 2 * cz + 4];
            }
            v = s * kI36;
            if (yy >= 0 && yy < nr) v += -sb.qr[y + 8][c + 4] * (1.0 / (yy + 0.5));
        }
        sb.g[y + 6][c + 2] = v;
    }
    for (int k = t; k < S::HH * RZ; k += NT) {
        const int y = k / RZ - 6, c = k % RZ, yy = r0 + y;
        double v = 0.0;
        if (yy >= 0 && yy < nr) {
            auto b = [&](int cc) { return sb.pz[y + 8][cc + 4]; };
            // forward: out(z) = (-in(z+2) + 8 in(z+1) - 8 in(z-1) + in(z-2)) / 12
            v = (-b(c - 2) + 8.0 * b(c - 1) - 8.0 * b(c + 1) + b(c + 2)) * (kI12 * kI18) * (1.0 / (yy + 0.5));
        }
        sb.h[y + 6][c] = v;
    }
}

// step 3 (after a barrier): psi-bar_B at region node (c, y), a real row
template <int RZ, int RH, bool kAxi>
__device__ __forceinline__ double psibar_at(const PsiBar<RZ, RH>& sb, int c, int y, int r0, int nr) {
    auto real = [&](int yy) { return r0 + yy >= 0 && r0 + yy < nr; };
    // psi-bar of extended row e at this column (before folding)
    auto ext = [&](int e) {
        const int y = e - r0;
        double s = 0.0;
        if (kAxi) {
            // d_r psi = isotropic d_r of the extended psi; only the rows
            // -2 .. nr + 1 carry an adjoint
#pragma unroll
            for (int i = 1; i < lbm::kQ; ++i) {
                const int cr = lbm::cr(i), cz = lbm::cz(i);
                if (cr == 0) continue;
                const int y1 = y - cr, y2 = y - 2 * cr;
                if (r0 + y1 >= -2 && r0 + y1 < nr + 2) s += (8.0 * cr / 36.0) * sb.g[y1 + 6][c - cz + 2];
                if (r0 + y2 >= -2 && r0 + y2 < nr + 2) s -= (cr / 36.0) * sb.g[y2 + 6][c - 2 * cz + 2];
            }
            // 1D d_r psi on real rows: (-p(y+2) + 8 p(y+1) - 8 p(y-1) + p(y-2)) / 12
            const int ys[4] = {y - 2, y - 1, y + 1, y + 2};
            const double cf[4] = {-1.0, 8.0, -8.0, 1.0};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (real(ys[k])) s += (cf[k] / 12.0) * sb.h[ys[k] + 6][c];
        }
        // Shan–Chen force: F^SC(x) = -G psi(x) sum_i W_i psi(x + c_i) c_i
#pragma unroll
        for (int i = 1; i < lbm::kQ; ++i) {
            const int ysrc = y - lbm::cr(i), cs = c - lbm::cz(i);
            if (real(ysrc))
                s += lbm::weight(i) * (lbm::cz(i) * sb.pz[ysrc + 8][cs + 4] + lbm::cr(i) * sb.pr[ysrc + 8][cs + 4]);
        }
        return s;
    };
    const int r = r0 + y;
    double psib = ext(r);
    if (r <= 3) psib += ext(-1 - r);            // axis images (rows -4 .. -1)
    if (r >= nr - 4) psib += ext(2 * nr - 1 - r);  // wall images (rows nr .. nr + 3)
    return psib;
}

// Kernel A.  kAxi: the axisymmetric terms (source, F^{sym}, velocity
// stencils) on; off, the plain 2D Shan–Chen step.
// kFused (small lattices): rho-bar_B of lam^{t+1} is not read but formed
// here, from the previous reverse step's P and E, on the tile and a 3-node
// ring (the gathers' targets), so that a run needs no kernel B between its
// steps; the gathered nu then completes in a step 3b, after the velocities.
// The 256-thread instance is held to three waves per SIMD (168 VGPRs), so
// that three workgroups share a CU and their loads overlap each other's
// arithmetic.
template <int TZ, int TR, bool kAxi, int NT, bool kFused>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 256 ? 3 : 1))) void adj_tile_a(const TileArgs a) {
    using T = Tile<TZ, TR, NT>;
    // kFused: the region of tile and 3-node ring
    constexpr int RZ = kFused ? TZ + 6 : 1, RH = kFused ? TR + 6 : 1;
    static_assert(!kFused || RZ * RH <= NT, "one region node per thread");
    __shared__ double s_psi[T::PH][T::PW];
    __shared__ double s_dr[T::DH][T::DW];
    __shared__ double s_d1[T::EH][T::EW];
    __shared__ double s_uz[T::UH][T::UW];
    __shared__ double s_ur[T::UH][T::UW];
    // adjoints of the velocity stencils: s_hz of d_r u_z and of d_z u_r
    // (equal), s_hr of d_r u_r
    __shared__ double s_hz[T::UH][T::UW];
    __shared__ double s_hr[T::UH][T::UW];
    __shared__ double s_red[2][NT / 64];
    __shared__ PsiBar<RZ, RH> sb;  // kFused: psi-bar_B of lam^{t+1} on the region
    __shared__ double s_rb[RH][RZ];  // kFused: rho-bar_B of lam^{t+1} on the region

    const int tile = block_tile(blockIdx.x, gridDim.x, a.tiles_z);
    const int z0 = (tile % a.tiles_z) * TZ, r0 = (tile / a.tiles_z) * TR;
    const int nz = a.nz, nr = a.nr;
    const size_t n = (size_t)a.n;
    const int t = threadIdx.x, tc = t % TZ, ty = t / TZ;
    const double G = a.G, tau = a.tau, rho0 = a.rho0;
    const double mu_f = (tau - 0.5) / 3.0, inv_rho0 = 1.0 / rho0;
    const Bufs bf = bufs_of(a);
    const bool has_p = kFused && a.pz_in != nullptr;

    // ---- 1. loads: psi on the window; nu, and the velocity-stencil
    // adjoints, within 2 of the tile
    auto psi_of = [&](double rho) { return rho0 * (1.0 - exp(-rho * inv_rho0)); };
    auto store_h = [&](int c, int y, bool real, double rho, double hz, double hr) {
        if (kAxi) {
            const double mu_r = rho * mu_f / (r0 + y + 0.5);
            s_hz[y + 2][c + 2] = real ? hz * mu_r : 0.0;
            s_hr[y + 2][c + 2] = real ? 2.0 * hr * mu_r : 0.0;
        }
    };
    const int zt = wrap_col(z0 + tc, nz), rt = r0 + ty;
    const bool has_tile = NT == T::NTILE || t < T::NTILE;  // a thread with a tile node
    const bool real_t = has_tile && rt < nr;
    const bool active = real_t && z0 + tc < nz;
    double rho_t = 0, jz_t = 0, jr_t = 0, nuf_t = 0;
    double nu[lbm::kQ];  // the tile node's nu, kept to step 4 (a reload there misses L2)
    double fk[lbm::kQ];  // kFused: the tile node's populations, kept to step 3b
    const unsigned xt = 8u * (unsigned)(mirror_even(rt, nr) * nz + zt);
    if (has_tile) {
        double fl[lbm::kQ];
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) fl[i] = ld(bf.f, xt, i * bf.plane);
        // a ghost row (last tile of a short lattice) gathers at the last
        // row and discards the values: no branch around the loads
        const int rg = real_t ? rt : nr - 1;
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) {
            const double v = gather_nu(a, bf, i, zt, rg);
            nu[i] = real_t ? v : 0.0;
        }
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) {
            rho_t += fl[i];
            jz_t += lbm::cz(i) * fl[i];
            jr_t += lbm::cr(i) * fl[i];
            if (!kFused) nuf_t += nu[i] * fl[i];  // sum_i nu_i f_i, the populations' part of tau-bar
            if (kFused) fk[i] = fl[i];
        }
        s_psi[ty + 6][tc + 6] = psi_of(rho_t);
        if (!kFused) {
            double hz = 0, hr = 0;
#pragma unroll
            for (int i = 0; i < lbm::kQ; ++i) {
                hz += 3.0 * lbm::weight(i) * lbm::cz(i) * nu[i];
                hr += 3.0 * lbm::weight(i) * lbm::cr(i) * nu[i];
            }
            store_h(tc, ty, real_t, rho_t, hz, hr);
        }
    }
    // the tile node's loads are consumed before the ring's are issued (all of
    // them at once do not fit the registers of the large-lattice instance)
    __builtin_amdgcn_sched_barrier(0);
    // ring nodes; the first slot's node, when within 2 of the tile, keeps
    // rho and j for its velocity
    double rho_q = 0, jz_q = 0, jr_q = 0;
    double vq[lbm::kQ - 1];  // kFused: the gathered lam_p of that node, kept to step 3b
    int cq = 0, yq = 0;
    const bool ring2 = t < T::R2N;
#pragma unroll
    for (int s = 0; s < T::RS; ++s) {
        const int k = t + s * NT;
        // every slot loads (a slot past the ring reads some lattice node and
        // stores nothing): no branch around the loads
        int c, y;
        ring_pos<TZ, TR>(k, c, y);
        const int z = wrap_col(z0 + c, nz), yy = r0 + y;
        const unsigned x = 8u * (unsigned)(mirror_even(yy, nr) * nz + z);
        double fr[lbm::kQ];
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) fr[i] = ld(bf.f, x, i * bf.plane);
        if (k < T::R2N + T::OUTN) {
            double rho = 0, jz = 0, jr = 0;
#pragma unroll
            for (int i = 0; i < lbm::kQ; ++i) {
                rho += fr[i];
                jz += lbm::cz(i) * fr[i];
                jr += lbm::cr(i) * fr[i];
            }
            s_psi[y + 6][c + 6] = psi_of(rho);
            if (s == 0 && ring2) {
                rho_q = rho;
                jz_q = jz;
                jr_q = jr;
                cq = c;
                yq = y;
                if (kAxi) {
                    // ghost rows gather at a clamped row and store 0
                    const bool real = yy >= 0 && yy < nr;
                    const int yg = yy < 0 ? 0 : (yy >= nr ? nr - 1 : yy);
                    double hz = 0, hr = 0;
#pragma unroll
                    for (int i = 1; i < lbm::kQ; ++i) {
                        const double v = gather_nu(a, bf, i, z, yg);
                        if (kFused) vq[i - 1] = v;
                        hz += 3.0 * lbm::weight(i) * lbm::cz(i) * v;
                        hr += 3.0 * lbm::weight(i) * lbm::cr(i) * v;
                    }
                    if (!kFused) store_h(c, y, real, rho, hz, hr);
                }
            }
        }
    }
    // kFused: P of lam^{t+1} on the region's window, and E at the thread's
    // region node
    double e_q = 0.0;
    if (kFused && has_p) {
        psibar_load<RZ, RH, NT, kAxi>(sb, a.pz_in, a.pr_in, n * sizeof(double), z0 - 3, r0 - 3, nz, nr, t);
        const int c = t % RZ - 3, y = t / RZ - 3;
        e_q = ld(rsrc_of(a.ex_in, n * sizeof(double)), 8u * (unsigned)((r0 + y) * nz + wrap_col(z0 + c, nz)), 0u);
    }
    __syncthreads();

    // ---- 2. d_r psi (isotropic, on the extended rows as they come) and the
    // 1D fourth-order d_r psi that d_zr differences along z (Sec. II.D)
    auto P = [&](int c, int y) { return s_psi[y + 6][c + 6]; };
    if (kAxi) {
        for (int k = t; k < T::DH * T::DW; k += NT) {
            const int y = k / T::DW - 4, c = k % T::DW - 4;
            double s = 0.0;
#pragma unroll
            for (int i = 1; i < lbm::kQ; ++i) {
                const int cr = lbm::cr(i), cz = lbm::cz(i);
                if (cr == 0) continue;
                s += cr * (8.0 * P(c + cz, y + cr) - P(c + 2 * cz, y + 2 * cr));
            }
            s_dr[y + 4][c + 4] = s * kI36;
        }
        for (int k = t; k < T::EH * T::EW; k += NT) {
            const int y = k / T::EW - 2, c = k % T::EW - 4;
            s_d1[y + 2][c + 4] = (-P(c, y + 2) + 8.0 * P(c, y + 1) - 8.0 * P(c, y - 1) + P(c, y - 2)) * kI12;
        }
        if (kFused && has_p) psibar_stencils<RZ, RH, NT>(sb, r0 - 3, nr, t);
        __syncthreads();
    }

    // ---- 3. force and velocity (Eqs. scforce, uhydro) at window node
    // (c, y), a real node; ghost rows of the velocity window take their
    // mirror node's velocity, u_r odd at the axis
    struct Fwd {
        double psi, sz, sr, dzr, drr, dr1, Fz, Fr, uz, ur;
    };
    auto forward_at = [&](int c, int y, double rho, double jz, double jr) {
        Fwd o;
        o.psi = P(c, y);
        double sz = 0, sr = 0;
#pragma unroll
        for (int i = 1; i < lbm::kQ; ++i) {
            const double ps = P(c + lbm::cz(i), y + lbm::cr(i));
            sz += lbm::weight(i) * ps * lbm::cz(i);
            sr += lbm::weight(i) * ps * lbm::cr(i);
        }
        o.sz = sz;
        o.sr = sr;
        double Fz = -G * o.psi * sz, Fr = -G * o.psi * sr;
        o.dzr = o.drr = o.dr1 = 0.0;
        if (kAxi) {
            auto D1 = [&](int cc) { return s_d1[y + 2][cc + 4]; };
            o.dzr = (-D1(c + 2) + 8.0 * D1(c + 1) - 8.0 * D1(c - 1) + D1(c - 2)) * kI12;
            double s = 0.0;
#pragma unroll
            for (int i = 1; i < lbm::kQ; ++i) {
                const int cr = lbm::cr(i), cz = lbm::cz(i);
                if (cr == 0) continue;
                s += cr * (8.0 * s_dr[y + cr + 4][c + cz + 4] - s_dr[y + 2 * cr + 4][c + 2 * cz + 4]);
            }
            o.drr = s * kI36;
            o.dr1 = s_dr[y + 4][c + 4];
            const double ir = 1.0 / (r0 + y + 0.5);
            Fz += -(G * kI18) * o.psi * o.dzr * ir;
            Fr += -(G * kI18) * o.psi * (o.drr - o.dr1 * ir) * ir;
        }
        Fz += rho * a.gz;
        o.Fz = Fz;
        o.Fr = Fr;
        const double irho = 1.0 / rho;
        o.uz = (jz + 0.5 * Fz) * irho;
        o.ur = (jr + 0.5 * Fr) * irho;
        return o;
    };
    // where window node (c, y) of the velocity window takes its velocity: a
    // real row its own; rows -2, -1 and nr, nr + 1 their mirror node's (whose
    // populations the load read), u_r odd at the axis; rows further out are
    // never read by a tile node (*use false: u = 0).  One forward_at per slot.
    auto source_row = [&](int y, bool& use, double& sgn) {
        const int yy = r0 + y;
        use = yy >= -2 && yy < nr + 2;
        sgn = yy < 0 ? -1.0 : 1.0;
        if (yy >= 0 && yy < nr) return y;
        const int ym = (yy < 0 ? -1 - yy : 2 * nr - 1 - yy) - r0;
        return use ? ym : y;
    };
    Fwd fw{};
    {
        bool use;
        double sgn;
        const int ys = source_row(ty, use, sgn);
        if (has_tile && use) {
            const Fwd o = forward_at(tc, ys, rho_t, jz_t, jr_t);
            if (real_t) fw = o;
            if (kAxi) {
                s_uz[ty + 2][tc + 2] = o.uz;
                s_ur[ty + 2][tc + 2] = sgn * o.ur;
            }
        } else if (kAxi && has_tile) {
            s_uz[ty + 2][tc + 2] = 0.0;
            s_ur[ty + 2][tc + 2] = 0.0;
        }
    }
    if (kAxi && ring2) {
        bool use;
        double sgn;
        const int ys = source_row(yq, use, sgn);
        double uz = 0.0, ur = 0.0;
        if (use) {
            const Fwd o = forward_at(cq, ys, rho_q, jz_q, jr_q);
            uz = o.uz;
            ur = sgn * o.ur;
        }
        s_uz[yq + 2][cq + 2] = uz;
        s_ur[yq + 2][cq + 2] = ur;
    }
    // kFused: rho-bar_B of lam^{t+1} at the thread's region node (0 on rows
    // off the lattice, which no gather reads)
    if (kFused && t < RZ * RH) {
        const int c = t % RZ - 3, y = t / RZ - 3, yy = r0 + y;
        double rb = 0.0;
        if (has_p && yy >= 0 && yy < nr) rb = mul_rounded(psibar_at<RZ, RH, kAxi>(sb, c + 3, y + 3, r0 - 3, nr), e_q);
        s_rb[y + 3][c + 3] = rb;
    }
    if (kAxi || kFused) __syncthreads();

    // ---- 3b (kFused). nu = lam_p + rho-bar_B at the gathers' targets, then
    // the velocity-stencil adjoints and the populations' part of tau-bar, in
    // the order of step 1 of the unfused kernel
    if (kFused) {
        if (has_tile) {
            if (real_t) {
#pragma unroll
                for (int i = 0; i < lbm::kQ; ++i) {
                    int dc, dr;
                    push_offset(i, rt, nr, a.wall, dc, dr);
                    nu[i] = nu[i] + s_rb[ty + dr + 3][tc + dc + 3];
                }
            }
            double hz = 0, hr = 0;
#pragma unroll
            for (int i = 0; i < lbm::kQ; ++i) {
                nuf_t += nu[i] * fk[i];
                hz += 3.0 * lbm::weight(i) * lbm::cz(i) * nu[i];
                hr += 3.0 * lbm::weight(i) * lbm::cr(i) * nu[i];
            }
            store_h(tc, ty, real_t, rho_t, hz, hr);
        }
        if (kAxi && ring2) {
            const int yy = r0 + yq;
            const bool real = yy >= 0 && yy < nr;
            double hz = 0, hr = 0;
            if (real) {
#pragma unroll
                for (int i = 1; i < lbm::kQ; ++i) {
                    int dc, dr;
                    push_offset(i, yy, nr, a.wall, dc, dr);
                    const double v = vq[i - 1] + s_rb[yq + dr + 3][cq + dc + 3];
                    hz += 3.0 * lbm::weight(i) * lbm::cz(i) * v;
                    hr += 3.0 * lbm::weight(i) * lbm::cr(i) * v;
                }
            }
            store_h(cq, yq, real, rho_q, hz, hr);
        }
        if (kAxi) __syncthreads();
    }

    // ---- 4. the tile node: collision, equilibrium and source reversed,
    // the velocity-stencil adjoints of the neighbours folded in, velocity
    // and force reversed
    double g_node = 0.0, t_node = 0.0;
    if (active) {
        const int r = rt;
        const double rho = rho_t, rr = r + 0.5, ir = 1.0 / rr, irho = 1.0 / rho;
        const double inv_tau = 1.0 / tau;
        const double uz = fw.uz, ur = fw.ur, Fz = fw.Fz, Fr = fw.Fr;
        const double qz = (jz_t + tau * Fz) * irho, qr = (jr_t + tau * Fr) * irho;
        // the transposed velocity stencils first (LDS reads only), then the
        // velocity derivatives, each finished before the next part starts so
        // that their LDS reads are not all in flight at once
        double tz_b = 0.0, tr_b = 0.0;
        if (kAxi) {
            // transposed velocity stencils: the adjoints at the nodes whose
            // stencils read this node's velocity, at its own row and at its
            // ghost images (row -1 - r at the axis, u_r odd; row 2 nr - 1 - r
            // at the wall), rows outside the lattice holding none
            auto H = [&](const double (*s)[T::UW], int y, int dc) {
                const int yy = r0 + y;
                const double m = (yy >= 0 && yy < nr) ? 1.0 : 0.0;
                const int yl = y < -2 ? -2 : (y > TR + 1 ? TR + 1 : y);
                return m * s[yl + 2][tc + dc + 2];
            };
            auto gather = [&](int e, double sgn_r) {
                const int y = e - r0;
                double gz = 0, gzr = 0, grr = 0;
#pragma unroll
                for (int i = 1; i < lbm::kQ; ++i) {
                    const int cz = lbm::cz(i), cr = lbm::cr(i);
                    if (cr != 0) {
                        gz += 8.0 * cr * H(s_hz, y - cr, -cz);
                        gz -= cr * H(s_hz, y - 2 * cr, -2 * cz);
                        grr += 8.0 * cr * H(s_hr, y - cr, -cz);
                        grr -= cr * H(s_hr, y - 2 * cr, -2 * cz);
                    }
                    if (cz != 0) {
                        gzr += 8.0 * cz * H(s_hz, y - cr, -cz);
                        gzr -= cz * H(s_hz, y - 2 * cr, -2 * cz);
                    }
                }
                tz_b += gz * kI36;
                tr_b += sgn_r * (gzr + grr) * kI36;
            };
            gather(r, 1.0);
            if (r <= 1) gather(-1 - r, -1.0);
            if (r >= nr - 2) gather(2 * nr - 1 - r, 1.0);
        }
        __builtin_amdgcn_sched_barrier(0);
        double druz = 0, dzur = 0, drur = 0;
        if (kAxi) {
            auto U = [&](const double (*s)[T::UW], int dc, int dy) { return s[ty + dy + 2][tc + dc + 2]; };
            double a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
            for (int i = 1; i < lbm::kQ; ++i) {
                const int cz = lbm::cz(i), cr = lbm::cr(i);
                if (cr != 0) {
                    a1 += cr * (8.0 * U(s_uz, cz, cr) - U(s_uz, 2 * cz, 2 * cr));
                    a3 += cr * (8.0 * U(s_ur, cz, cr) - U(s_ur, 2 * cz, 2 * cr));
                }
                if (cz != 0) a2 += cz * (8.0 * U(s_ur, cz, cr) - U(s_ur, 2 * cz, 2 * cr));
            }
            druz = a1 * kI36;
            dzur = a2 * kI36;
            drur = a3 * kI36;
        }
        __builtin_amdgcn_sched_barrier(0);
        // tau-bar of BGK: sum_i nu_i (f_i - f^eq_i) / tau^2, its population
        // part summed in step 1 (the populations are not kept)
        double nfeq = 0.0;
        double rhob = 0, qzb = 0, qrb = 0, taub = 0, massb = 0, hzb = 0, hrb = 0;
        const double qq = 1.5 * (qz * qz + qr * qr);
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) {
            const double v = nu[i];
            const double wi = lbm::weight(i);
            const double cu = lbm::cz(i) * qz + lbm::cr(i) * qr;
            const double poly = 3.0 * cu + 4.5 * cu * cu - qq;
            const double feq = wi * rho * (1.0 + poly);
            nfeq += v * feq;
            const double feqb = v * inv_tau;
            rhob += feqb * wi * (1.0 + poly);
            const double dpoly = wi * rho * feqb * (3.0 + 9.0 * cu);  // d feq / d cu
            qzb += dpoly * lbm::cz(i) - feqb * wi * rho * 3.0 * qz;
            qrb += dpoly * lbm::cr(i) - feqb * wi * rho * 3.0 * qr;
            massb += wi * v;
            hzb += 3.0 * wi * lbm::cz(i) * v;
            hrb += 3.0 * wi * lbm::cr(i) * v;
        }
        taub += (nuf_t - nfeq) * inv_tau * inv_tau;
        double uzb = 0, urb = 0;
        if (kAxi) {
            const double mu = rho * (tau - 0.5) / 3.0;
            // mass = -rho u_r / r
            rhob += -massb * ur * ir;
            urb += -massb * rho * ir;
            // H_z = (mu (d_r u_z + d_z u_r) - rho u_r u_z) / r
            double mub = hzb * (druz + dzur) * ir;
            rhob += -hzb * ur * uz * ir;
            urb += -hzb * rho * uz * ir;
            uzb += -hzb * rho * ur * ir;
            // H_r = (2 mu (d_r u_r - u_r / r) - rho u_r^2) / r
            mub += hrb * 2.0 * (drur - ur * ir) * ir;
            urb += hrb * (-2.0 * mu * ir * ir - 2.0 * rho * ur * ir);
            rhob += -hrb * ur * ur * ir;
            // mu = rho (tau - 1/2) / 3
            rhob += mub * (tau - 0.5) / 3.0;
            taub += mub * rho / 3.0;
        }
        // u^eq = (j + tau F) / rho
        double jzb = qzb * irho, jrb = qrb * irho;
        double Fzb = tau * qzb * irho, Frb = tau * qrb * irho;
        taub += (qzb * Fz + qrb * Fr) * irho;
        rhob += -(qzb * qz + qrb * qr) * irho;
        if (kAxi) {
            uzb += tz_b;
            urb += tr_b;
        }
        // u = (j + F/2) / rho
        jzb += uzb * irho;
        jrb += urb * irho;
        Fzb += 0.5 * uzb * irho;
        Frb += 0.5 * urb * irho;
        rhob += -(uzb * uz + urb * ur) * irho;
        // F = F^SC + F^sym + rho g z^
        rhob += Fzb * a.gz;
        double Gb = -fw.psi * (Fzb * fw.sz + Frb * fw.sr);
        double psib = -G * (Fzb * fw.sz + Frb * fw.sr);
        if (kAxi) {
            const double g18 = G * kI18;
            // F^sym_z = -(G/18) psi d_zr / r
            Gb += Fzb * (-fw.psi * fw.dzr * kI18 * ir);
            psib += Fzb * (-g18 * fw.dzr * ir);
            // F^sym_r = -(G/18) psi (d_rr / r - d_r / r^2)
            const double br = (fw.drr - fw.dr1 * ir) * ir;
            Gb += Frb * (-fw.psi * br * kI18);
            psib += Frb * (-g18 * br);
        }
        // psi = rho0 (1 - exp(-rho / rho0)): the node's own psi-bar
        const double e = exp(-rho * inv_rho0);
        rhob += psib * e;
        const unsigned x = 8u * (unsigned)(rt * nz + zt);
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i)
            st(bf.out, x, i * bf.plane, nu[i] * (1.0 - inv_tau) + rhob + lbm::cz(i) * jzb + lbm::cr(i) * jrb);
        st(bf.pz, x, 0u, -G * fw.psi * Fzb);
        st(bf.pr, x, 0u, -G * fw.psi * Frb);
        st(bf.ex, x, 0u, e);
        g_node = Gb;
        t_node = taub;
    }
    // the tile's dL/dG and dL/dtau: a tree of lane shuffles per wave, then
    // the waves in order (a fixed order)
#pragma unroll
    for (int k = 32; k > 0; k >>= 1) {
        g_node += __shfl_down(g_node, k, 64);
        t_node += __shfl_down(t_node, k, 64);
    }
    if ((t & 63) == 0) {
        s_red[0][t >> 6] = g_node;
        s_red[1][t >> 6] = t_node;
    }
    __syncthreads();
    if (t == 0) {
        double g = 0.0, q = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            g += s_red[0][w];
            q += s_red[1][w];
        }
        double* o = a.part + 2 * (size_t)tile;
        if (a.accumulate) {
            o[0] += g;
            o[1] += q;
        } else {
            o[0] = g;
            o[1] = q;
        }
    }
}

// Kernel B: psi-bar from the psi stencils of the other nodes, through P.
// kFinal: add rho-bar_B to lam_out in every direction (lam_out then holds
// lam^t); otherwise write rho-bar_B.
template <int TZ, int TR, bool kAxi, bool kFinal, int NT>
__global__ __launch_bounds__(NT) void adj_tile_b(const TileArgs a) {
    __shared__ PsiBar<TZ, TR> sb;
    const int tile = block_tile(blockIdx.x, gridDim.x, a.tiles_z);
    const int z0 = (tile % a.tiles_z) * TZ, r0 = (tile / a.tiles_z) * TR;
    const int nz = a.nz, nr = a.nr;
    const int t = threadIdx.x, tc = t % TZ, ty = t / TZ;
    const size_t nb = (size_t)a.n * sizeof(double);
    psibar_load<TZ, TR, NT, kAxi>(sb, a.pz, a.pr, nb, z0, r0, nz, nr, t);
    __syncthreads();
    if (kAxi) {
        psibar_stencils<TZ, TR, NT>(sb, r0, nr, t);
        __syncthreads();
    }
    const int r = r0 + ty;
    if (t >= TZ * TR || r >= nr || z0 + tc >= nz) return;
    const double psib = psibar_at<TZ, TR, kAxi>(sb, tc, ty, r0, nr);
    const unsigned x = 8u * (unsigned)(r * nz + z0 + tc);
    // a rounded product, never fused into the additions below: a run adds
    // the stored rho-bar_B in the next step's gathers, and its lam must equal
    // that of single steps bit for bit
    const double rhob = mul_rounded(psib, ld(rsrc_of(a.ex, nb), x, 0u));
    if (kFinal) {
        // every load before the first store (the compiler cannot tell that
        // the stores do not alias them)
        const Rsrc ro = rsrc_of(a.lam_out, 9 * nb);
        double l[lbm::kQ];
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) l[i] = ld(ro, x, i * (unsigned)nb);
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) st(ro, x, i * (unsigned)nb, l[i] + rhob);
    } else {
        st(rsrc_of(a.rhob_out, nb), x, 0u, rhob);
    }
}

// acc[0] += dL/dG, acc[1] += dL/dtau: the block partials (of one step, or
// the running sums of a run) summed in a fixed order
__global__ void rev_reduce(const double* __restrict__ part, int nparts, double* acc) {
    __shared__ double s[2][256];
    const int t = threadIdx.x;
    double g = 0.0, q = 0.0;
    for (int b = t; b < nparts; b += 256) {
        g += part[2 * (size_t)b];
        q += part[2 * (size_t)b + 1];
    }
    s[0][t] = g;
    s[1][t] = q;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (t < k) {
            s[0][t] += s[0][t + k];
            s[1][t] += s[1][t + k];
        }
        __syncthreads();
    }
    if (t == 0) {
        acc[0] += s[0][0];
        acc[1] += s[1][0];
    }
}

// initial condition f_i = f^eq_i(rho0, u0): rho0-bar = sum_i lam_i d f^eq_i / d rho
__global__ void init_vjp_kernel(const double* lam, const double* uz, const double* ur, long long n, double* rho_bar) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const double vz = uz ? uz[x] : 0.0, vr = ur ? ur[x] : 0.0;
    const double qq = 1.5 * (vz * vz + vr * vr);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) {
        const double cu = lbm::cz(i) * vz + lbm::cr(i) * vr;
        s += lam[i * n + x] * lbm::weight(i) * (1.0 + 3.0 * cu + 4.5 * cu * cu - qq);
    }
    rho_bar[x] = s;
}

// density of a state [9][n] (for the loss observable)
__global__ void density_kernel(const double* f, long long n, double* rho) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) s += f[i * n + x];
    rho[x] = s;
}

// r_m = sum_k w_mk phi(node_k), phi = (rho - rho_g)/(rho_l - rho_g); one
// workgroup per probe row, fixed-order reduction
__global__ void ray_forward_kernel(const double* rho, const int* row_ptr, const int* col, const double* val,
                                   double rho_l, double rho_g, double* out) {
    __shared__ double s[256];
    const int m = blockIdx.x, t = threadIdx.x;
    double acc = 0.0;
    for (int k = row_ptr[m] + t; k < row_ptr[m + 1]; k += 256) acc += val[k] * (rho[col[k]] - rho_g);
    s[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    if (t == 0) out[m] = s[0] / (rho_l - rho_g);
}

// lam_i(x) += sum_m rbar_m w_mx / (rho_l - rho_g) for every i, from the
// node-major (transposed) copy of the probe matrix
__global__ void ray_vjp_kernel(const double* rbar, const int* node_ptr, const int* node_row, const double* node_val,
                               const int* nodes, int n_nodes, double rho_l, double rho_g, long long n, double* lam) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    double s = 0.0;
    for (int j = node_ptr[k]; j < node_ptr[k + 1]; ++j) s += rbar[node_row[j]] * node_val[j];
    s /= (rho_l - rho_g);
    const long long x = nodes[k];
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) lam[i * n + x] += s;
}

// loss += sum_m (r_m - target_m)^2 and rbar_m = 2 (r_m - target_m)
__global__ void misfit_kernel(const double* r, const double* target, int m, double* loss, double* rbar) {
    __shared__ double s[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int k = t; k < m; k += 256) {
        const double d = r[k] - target[k];
        if (rbar) rbar[k] = 2.0 * d;
        acc += d * d;
    }
    s[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    if (t == 0) *loss += s[0];
}

inline int nblk(long long n) { return (int)((n + 255) / 256); }

__global__ void zero_kernel(double* p, long long n) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = 0.0;
}


// Tile shapes.  Lattices with at least 192 tiles of 16 x 16 nodes (three
// for every four CUs): 16 x 16 nodes and 256 threads, three workgroups per
// CU (held to 168 VGPRs), kernels A and B per step.  At 2048 x 1024 the
// (forward + backward) / forward ratio was 5.40 with this shape, against
// 5.53 for 32 x 8 tiles (256 threads), 5.93 for 32 x 16 (512 threads, one
// workgroup per CU at 148 VGPRs), 6.26 for 32 x 8 (512 threads) and 6.33
// for 32 x 16 held to 128 VGPRs (spills); at 512 x 256, 384 x 192 and
// 362 x 181 it was 4.62, 4.39 and 4.35, against 6.82, 5.49 and 5.51 on the
// small-lattice path.  Smaller lattices (the 256 x 128 adjoint workload has
// 128 such tiles): 16 x 8 nodes with 512 threads, where a kernel's time is
// one workgroup's chain of loads and the spare threads share the window,
// and kernel B fused into the next step's kernel A (before the fusion, the
// reverse step took 19.5 us with 128 threads, 18.8 with 256, 18.6 with
// 512; 16 x 4 and 8 x 8 tiles were no faster with 256 threads and 25%
// slower with 512).
struct Shape {
    int tz, tr;
};
constexpr int kSmallTZ = 16, kSmallTR = 8, kSmallNT = 512;
constexpr int kLargeTZ = 16, kLargeTR = 16, kLargeNT = 256;
Shape shape_of(int nz, int nr) {
    const long long large = (long long)((nz + kLargeTZ - 1) / kLargeTZ) * ((nr + kLargeTR - 1) / kLargeTR);
    return large >= 192 ? Shape{kLargeTZ, kLargeTR} : Shape{kSmallTZ, kSmallTR};
}
long long tiles_of(int nz, int nr) {
    const Shape s = shape_of(nz, nr);
    return (long long)((nz + s.tz - 1) / s.tz) * ((nr + s.tr - 1) / s.tr);
}

// workspace (doubles): rho-bar_B [n]; two sets of P_z, P_r, E [n] each
// (the fused kernel A reads the previous step's set while it writes its
// own); the tiles' partial sums of one step [tiles][2]; the running sums of
// a run [tiles][2]
constexpr size_t kWsFields = 7;
struct Layout {
    double *rhob, *pz[2], *pr[2], *ex[2], *part, *run;
};
Layout layout_of(void* ws, int nz, int nr) {
    const size_t n = (size_t)nz * nr;
    const size_t nt = (size_t)tiles_of(nz, nr);
    double* b = static_cast<double*>(ws);
    Layout w;
    w.rhob = b;
    for (int k = 0; k < 2; ++k) {
        w.pz[k] = b + (1 + 3 * k) * n;
        w.pr[k] = b + (2 + 3 * k) * n;
        w.ex[k] = b + (3 + 3 * k) * n;
    }
    w.part = b + kWsFields * n;
    w.run = w.part + 2 * nt;
    return w;
}

TileArgs tile_args(const lbm_axi_params* p, const Layout& w) {
    TileArgs a{};
    a.nz = p->nz;
    a.nr = p->nr;
    a.n = (long long)p->nz * p->nr;
    a.G = p->G;
    a.tau = p->tau;
    a.rho0 = p->psi_rho0;
    a.gz = p->gz;
    a.wall = p->wall;
    a.tiles_z = (p->nz + shape_of(p->nz, p->nr).tz - 1) / shape_of(p->nz, p->nr).tz;
    a.pz = w.pz[0];
    a.pr = w.pr[0];
    a.ex = w.ex[0];
    return a;
}

// the small-lattice path fuses kernel B into the next step's kernel A
bool fused_path(int nz, int nr) { return shape_of(nz, nr).tr != kLargeTR; }

template <int TZ, int TR, int NT, bool kFused>
void launch_a_t(const TileArgs& a, bool axi, int tiles, hipStream_t s) {
    if (axi)
        hipLaunchKernelGGL((adj_tile_a<TZ, TR, true, NT, kFused>), dim3(tiles), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((adj_tile_a<TZ, TR, false, NT, kFused>), dim3(tiles), dim3(NT), 0, s, a);
}
template <int TZ, int TR, int NT>
void launch_b_t(const TileArgs& a, bool axi, bool final, int tiles, hipStream_t s) {
    const dim3 g(tiles), b(NT);
    if (axi && final) hipLaunchKernelGGL((adj_tile_b<TZ, TR, true, true, NT>), g, b, 0, s, a);
    if (axi && !final) hipLaunchKernelGGL((adj_tile_b<TZ, TR, true, false, NT>), g, b, 0, s, a);
    if (!axi && final) hipLaunchKernelGGL((adj_tile_b<TZ, TR, false, true, NT>), g, b, 0, s, a);
    if (!axi && !final) hipLaunchKernelGGL((adj_tile_b<TZ, TR, false, false, NT>), g, b, 0, s, a);
}
void launch_a(const TileArgs& a, bool axi, hipStream_t s) {
    const int tiles = (int)tiles_of(a.nz, a.nr);
    if (fused_path(a.nz, a.nr))
        launch_a_t<kSmallTZ, kSmallTR, kSmallNT, true>(a, axi, tiles, s);
    else
        launch_a_t<kLargeTZ, kLargeTR, kLargeNT, false>(a, axi, tiles, s);
}
// final: lam^t complete in a.lam_out; otherwise its rho-bar_B part in
// a.rhob_out
void launch_b(const TileArgs& a, bool axi, bool final, hipStream_t s) {
    const int tiles = (int)tiles_of(a.nz, a.nr);
    if (fused_path(a.nz, a.nr))
        launch_b_t<kSmallTZ, kSmallTR, kSmallNT>(a, axi, final, tiles, s);
    else
        launch_b_t<kLargeTZ, kLargeTR, kLargeNT>(a, axi, final, tiles, s);
}

// grids the reverse step handles: its psi window mirrors up to six rows at
// the axis and the wall (nz >= 4, nr >= 6), node indices of the window are
// 32-bit, and the kernels address a whole FP64 state (nine planes) through
// buffer resources with 32-bit byte offsets, so one state stays below 4 GiB
bool adjoint_grid_ok(int nz, int nr) {
    return nz >= 4 && nr >= 6 && (long long)nz * (nr + 12) <= INT_MAX &&
           9ull * 8ull * (unsigned long long)nz * (unsigned long long)nr < (1ull << 32);
}

int check_adjoint(const lbm_axi_params* p, size_t ws_bytes) {
    if (!p) return LBM_AXI_EINVAL;
    if (!adjoint_grid_ok(p->nz, p->nr) || !(p->tau > 0.5) || !(p->psi_rho0 > 0.0)) return LBM_AXI_EINVAL;
    if (p->wall != 0 && p->wall != 1) return LBM_AXI_EINVAL;
    if (p->precision != LBM_AXI_FP64 || p->flags != 0) return LBM_AXI_EUNSUP;
    if (ws_bytes < lbm_axi_adjoint_workspace_bytes(p->nz, p->nr)) return LBM_AXI_ENOMEM;
    return LBM_AXI_OK;
}

// one reverse step into d_lam with the workspace at ws (both public single
// steps)
int reverse_step(const lbm_axi_params* p, const double* d_f, const double* d_lam_next, double* d_lam,
                 double* d_grad_acc, void* ws, hipStream_t s) {
    const Layout w = layout_of(ws, p->nz, p->nr);
    TileArgs a = tile_args(p, w);
    a.f = d_f;
    a.lam_p = d_lam_next;
    a.rhob_in = nullptr;
    a.lam_out = d_lam;
    a.part = w.part;
    a.accumulate = 0;
    // kernel A (which, fused, finds no previous step's P: pz_in NULL), then
    // kernel B completing lam^t in place
    launch_a(a, p->axisym != 0, s);
    launch_b(a, p->axisym != 0, true, s);
    if (d_grad_acc)
        hipLaunchKernelGGL(rev_reduce, dim3(1), dim3(256), 0, s, w.part, (int)tiles_of(p->nz, p->nr), d_grad_acc);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_AXI_OK : lbm_host::hip_fail(e, "adjoint kernel launch");
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's scratch address, looked up once per device
int noalloc_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lbm_host::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return lbm_host::fail(LBM_AXI_EUNSUP, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return lbm_host::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return lbm_host::fail(LBM_AXI_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_AXI_OK;
}

}  // namespace

extern "C" {

int lbm_axi_adjoint_step_noalloc(const lbm_axi_params* p, const double* d_f, const double* d_lam_next, double* d_lam,
                                 double* d_grad_acc, void* hip_stream) {
    if (!p || !d_f || !d_lam_next || !d_lam) return lbm_host::fail(LBM_AXI_EINVAL, "NULL argument");
    const size_t need = lbm_axi_adjoint_workspace_bytes(p->nz, p->nr);
    if (need == 0) return lbm_host::fail(LBM_AXI_EINVAL, "invalid grid %d x %d for the adjoint", p->nz, p->nr);
    if (need > (size_t)LBM_AXI_NOALLOC_SCRATCH_BYTES)
        return lbm_host::fail(LBM_AXI_ENOMEM,
                              "grid %d x %d needs %zu bytes of scratch; the static scratch holds %zu "
                              "(use lbm_axi_adjoint_step with a workspace)",
                              p->nz, p->nr, need, (size_t)LBM_AXI_NOALLOC_SCRATCH_BYTES);
    const int rc = check_adjoint(p, need);
    if (rc != LBM_AXI_OK) return lbm_host::fail(rc, "adjoint parameters rejected (FP64, flags 0, tau > 1/2)");
    void* ws = nullptr;
    const int rs = noalloc_scratch(&ws);
    if (rs != LBM_AXI_OK) return rs;
    // the kernels write every field and partial sum of one step before
    // reading it, so nothing needs clearing
    return reverse_step(p, d_f, d_lam_next, d_lam, d_grad_acc, ws, static_cast<hipStream_t>(hip_stream));
}

size_t lbm_axi_adjoint_workspace_bytes(int32_t nz, int32_t nr) {
    if (!adjoint_grid_ok(nz, nr)) return 0;
    const size_t n = (size_t)nz * nr;
    return (kWsFields * n + 4 * (size_t)tiles_of(nz, nr)) * sizeof(double);
}

int lbm_axi_adjoint_step(const lbm_axi_params* p, const double* d_f, const double* d_lam_next, double* d_lam,
                         double* d_grad_acc, void* d_ws, size_t ws_bytes, void* hip_stream) {
    if (!p || !d_f || !d_lam_next || !d_lam || !d_ws) return LBM_AXI_EINVAL;
    const int rc = check_adjoint(p, ws_bytes);
    if (rc != LBM_AXI_OK) return rc;
    return reverse_step(p, d_f, d_lam_next, d_lam, d_grad_acc, d_ws, static_cast<hipStream_t>(hip_stream));
}

int lbm_axi_adjoint_run(const lbm_axi_params* p, const double* d_states, int32_t k, double* d_lam, double* d_tmp,
                        double* d_grad_acc, void* d_ws, size_t ws_bytes, void* hip_stream) {
    if (!p || !d_states || !d_lam || !d_tmp || d_tmp == d_lam || !d_ws || k < 0) return LBM_AXI_EINVAL;
    const int rc = check_adjoint(p, ws_bytes);
    if (rc != LBM_AXI_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t n9 = 9 * (size_t)p->nz * (size_t)p->nr;
    const Layout w = layout_of(d_ws, p->nz, p->nr);
    const int tiles = (int)tiles_of(p->nz, p->nr);
    // the tiles' sums of dL/dG, dL/dtau run over the k steps and are reduced
    // once at the end (a kernel, not a memset, clears them)
    hipLaunchKernelGGL(zero_kernel, dim3(nblk(2 * (long long)tiles)), dim3(256), 0, s, w.run, 2 * (long long)tiles);
    double* cur = d_lam;  // lam^{t0+j+1} before step j: all of it (j = k - 1), or its lam_p part
    double* nxt = d_tmp;
    const bool fused = fused_path(p->nz, p->nr), axi = p->axisym != 0;
    for (int32_t j = k - 1; j >= 0; --j) {
        TileArgs a = tile_args(p, w);
        a.f = d_states + (size_t)j * n9;
        a.lam_p = cur;
        a.lam_out = nxt;
        a.rhob_out = w.rhob;
        a.part = w.run;
        a.accumulate = 1;
        if (fused) {
            // step j writes P and E to set j % 2 and forms the rest of
            // lam^{j+1} from set (j + 1) % 2; a kernel B only completes lam
            // after the last step
            const int mine = j & 1, prev = 1 - mine;
            a.pz = w.pz[mine];
            a.pr = w.pr[mine];
            a.ex = w.ex[mine];
            a.rhob_in = nullptr;
            a.pz_in = j == k - 1 ? nullptr : w.pz[prev];
            a.pr_in = j == k - 1 ? nullptr : w.pr[prev];
            a.ex_in = j == k - 1 ? nullptr : w.ex[prev];
            launch_a(a, axi, s);
            if (j == 0) launch_b(a, axi, true, s);
        } else {
            a.rhob_in = j == k - 1 ? nullptr : w.rhob;
            launch_a(a, axi, s);
            launch_b(a, axi, j == 0, s);
        }
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (d_grad_acc && k > 0) hipLaunchKernelGGL(rev_reduce, dim3(1), dim3(256), 0, s, w.run, tiles, d_grad_acc);
    if (hipGetLastError() != hipSuccess) return LBM_AXI_EHIP;
    if (cur != d_lam && hipMemcpyAsync(d_lam, cur, n9 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return LBM_AXI_EHIP;
    return LBM_AXI_OK;
}

int lbm_axi_init_vjp(const double* d_lam0, const double* d_uz0, const double* d_ur0, int32_t nz, int32_t nr,
                     double* d_rho0_bar, void* hip_stream) {
    if (!d_lam0 || !d_rho0_bar) return lbm_host::fail(LBM_AXI_EINVAL, "init_vjp: NULL argument");
    if (nz < 1 || nr < 1) return lbm_host::fail(LBM_AXI_EINVAL, "init_vjp: grid %d x %d", nz, nr);
    const long long n = (long long)nz * nr;
    hipLaunchKernelGGL(init_vjp_kernel, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_lam0,
                       d_uz0, d_ur0, n, d_rho0_bar);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_density(const double* d_f, int32_t nz, int32_t nr, double* d_rho, void* hip_stream) {
    if (!d_f || !d_rho) return lbm_host::fail(LBM_AXI_EINVAL, "density: NULL argument");
    if (nz < 1 || nr < 1) return lbm_host::fail(LBM_AXI_EINVAL, "density: grid %d x %d", nz, nr);
    const long long n = (long long)nz * nr;
    hipLaunchKernelGGL(density_kernel, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_f, n, d_rho);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_ray_forward(const double* d_rho, int32_t n_rows, const int32_t* d_row_ptr, const int32_t* d_col,
                        const double* d_val, double rho_l, double rho_g, double* d_out, void* hip_stream) {
    if (!d_rho || !d_row_ptr || !d_col || !d_val || !d_out)
        return lbm_host::fail(LBM_AXI_EINVAL, "ray_forward: NULL argument");
    if (n_rows < 0) return lbm_host::fail(LBM_AXI_EINVAL, "ray_forward: n_rows %d", n_rows);
    if (!std::isfinite(rho_l) || !std::isfinite(rho_g) || rho_l == rho_g)
        return lbm_host::fail(LBM_AXI_EINVAL, "ray_forward: rho_l and rho_g must be finite and differ");
    if (n_rows == 0) return LBM_AXI_OK;
    hipLaunchKernelGGL(ray_forward_kernel, dim3(n_rows), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_rho,
                       d_row_ptr, d_col, d_val, rho_l, rho_g, d_out);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_ray_vjp(const double* d_rbar, int32_t n_nodes, const int32_t* d_node_ptr, const int32_t* d_node_row,
                    const double* d_node_val, const int32_t* d_nodes, double rho_l, double rho_g, int32_t nz,
                    int32_t nr, double* d_lam, void* hip_stream) {
    if (!d_rbar || !d_node_ptr || !d_node_row || !d_node_val || !d_nodes || !d_lam)
        return lbm_host::fail(LBM_AXI_EINVAL, "ray_vjp: NULL argument");
    // the kernel adds into the nine planes of nz nr values of d_lam
    if (n_nodes < 0 || nz < 1 || nr < 1 || (long long)nz * nr > INT_MAX)
        return lbm_host::fail(LBM_AXI_EINVAL, "ray_vjp: n_nodes %d, grid %d x %d", n_nodes, nz, nr);
    if (!std::isfinite(rho_l) || !std::isfinite(rho_g) || rho_l == rho_g)
        return lbm_host::fail(LBM_AXI_EINVAL, "ray_vjp: rho_l and rho_g must be finite and differ");
    if (n_nodes == 0) return LBM_AXI_OK;
    hipLaunchKernelGGL(ray_vjp_kernel, dim3((n_nodes + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       d_rbar, d_node_ptr, d_node_row, d_node_val, d_nodes, n_nodes, rho_l, rho_g,
                       (long long)nz * nr, d_lam);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_misfit(const double* d_r, const double* d_target, int32_t m, double* d_loss, double* d_rbar,
                   void* hip_stream) {
    if (!d_r || !d_target || !d_loss) return lbm_host::fail(LBM_AXI_EINVAL, "misfit: NULL argument");
    if (m < 0) return lbm_host::fail(LBM_AXI_EINVAL, "misfit: m %d", m);
    hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_r, d_target, m,
                       d_loss, d_rbar);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_ray_weights(int32_t nz, int32_t nr, double zc, const double* h_thetas, int32_t n_rays, double ds,
                        double s_max, int32_t cap, int32_t* h_row_ptr, int32_t* h_col, double* h_val,
                        int32_t* h_node_ptr, int32_t* h_nodes, int32_t* h_node_row, double* h_node_val,
                        int32_t* h_nnz, int32_t* h_n_nodes) {
    using lbm_host::fail;
    if (nz < 1 || nr < 1 || n_rays < 0 || !h_nnz || !h_n_nodes || (n_rays > 0 && !h_thetas))
        return fail(LBM_AXI_EINVAL, "ray weights: need nz, nr >= 1, n_rays >= 0 and non-NULL outputs");
    if ((long long)nz * nr > INT_MAX) return fail(LBM_AXI_EINVAL, "ray weights: grid %d x %d too large", nz, nr);
    // the sample coordinates are converted to int: finite, and within
    // kMaxRayReach of the origin; at most kMaxRaySamples samples per ray
    constexpr double kMaxRayReach = 1e9;
    constexpr double kMaxRaySamples = 1 << 24;
    if (!std::isfinite(ds) || !(ds > 0.0) || !std::isfinite(s_max) || !(s_max >= 0.0) || !std::isfinite(zc))
        return fail(LBM_AXI_EINVAL, "ray weights: ds > 0, s_max >= 0 and zc must be finite");
    if (std::fabs(zc) + s_max > kMaxRayReach)
        return fail(LBM_AXI_EINVAL, "ray weights: |zc| + s_max beyond %g", kMaxRayReach);
    if (std::floor(s_max / ds) > kMaxRaySamples)
        return fail(LBM_AXI_EINVAL, "ray weights: s_max / ds gives more than %g samples per ray", kMaxRaySamples);
    for (int m = 0; m < n_rays; ++m)
        if (!std::isfinite(h_thetas[m])) return fail(LBM_AXI_EINVAL, "ray weights: theta %d is not finite", m);
    try {
        // per ray: node -> weight of the bilinear interpolants of the samples
        // s_k = (k + 1/2) ds along the ray from (zc, 0) at angle theta; rows
        // below row 0 mirror onto the real rows, rows above the last clamp to
        // it, z is periodic
        std::vector<std::map<int32_t, double>> rows((size_t)n_rays);
        const int nk = (int)std::floor(s_max / ds);
        for (int m = 0; m < n_rays; ++m) {
            const double ct = std::cos(h_thetas[m]), st = std::sin(h_thetas[m]);
            for (int k = 0; k < nk; ++k) {
                const double sk = (k + 0.5) * ds;
                const double zz = zc + sk * ct, y = sk * st - 0.5;
                const int j0 = (int)std::floor(y), k0 = (int)std::floor(zz);
                const double ty = y - j0, tz = zz - k0;
                for (int dj = 0; dj < 2; ++dj) {
                    const double wy = dj ? ty : 1.0 - ty;
                    int jj = j0 + dj;
                    if (jj < 0) jj = -1 - jj;
                    if (jj > nr - 1) jj = nr - 1;
                    for (int dk = 0; dk < 2; ++dk) {
                        const double wz = dk ? tz : 1.0 - tz;
                        const double wgt = ds * wy * wz;
                        if (wgt == 0.0) continue;
                        int kk = (k0 + dk) % nz;
                        if (kk < 0) kk += nz;
                        rows[m][jj * nz + kk] += wgt;
                    }
                }
            }
        }
        std::map<int32_t, std::vector<std::pair<int32_t, double>>> by_node;
        long long total = 0;
        for (int m = 0; m < n_rays; ++m) total += (long long)rows[m].size();
        if (total > INT_MAX) return fail(LBM_AXI_EINVAL, "ray weights: %lld entries, beyond 32-bit indices", total);
        const int32_t nnz = (int32_t)total;
        for (int m = 0; m < n_rays; ++m)
            for (const auto& kv : rows[m]) by_node[kv.first].push_back({m, kv.second});
        *h_nnz = nnz;
        *h_n_nodes = (int32_t)by_node.size();
        if (!h_row_ptr || !h_col || !h_val || !h_node_ptr || !h_nodes || !h_node_row || !h_node_val) return LBM_AXI_OK;
        if (cap < nnz) return fail(LBM_AXI_ENOMEM, "ray weights: capacity %d below nnz %d", cap, nnz);
        int32_t k = 0;
        h_row_ptr[0] = 0;
        for (int m = 0; m < n_rays; ++m) {
            for (const auto& kv : rows[m]) {
                h_col[k] = kv.first;
                h_val[k] = kv.second;
                ++k;
            }
            h_row_ptr[m + 1] = k;
        }
        int32_t j = 0, q = 0;
        h_node_ptr[0] = 0;
        for (const auto& kv : by_node) {
            h_nodes[q] = kv.first;
            for (const auto& e : kv.second) {
                h_node_row[j] = e.first;
                h_node_val[j] = e.second;
                ++j;
            }
            h_node_ptr[++q] = j;
        }
        return LBM_AXI_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_AXI_ENOMEM, "ray weights: host allocation failed");
    }
}

}  // extern "C"
