// Fused per-timestep kernel of the axisymmetric Shan–Chen lattice Boltzmann
// method (Srivastava et al., arXiv:1310.1871, Sec. II).
//
// One workgroup owns a TZ x TR tile of nodes and does, entirely on chip:
//   1. reads the post-streaming populations of the tile (kept in registers)
//      and of a 6-node halo, and forms rho, psi(rho) (Sec. II.A) into LDS;
//      halo rows below the axis and above the wall hold the mirrored values
//      (symmetry rule at the axis, zero-derivative rule at the wall,
//      Sec. II.E), columns wrap periodically;
//   2. the isotropic d_r psi on a 4-node halo (Sec. II.D, first stencil),
//      and the 1D fourth-order d_r psi that d_zr differences along z;
//   3. the total force F = F^SC (Eq. scforce) + F^{gamma,sym}
//      (Eq. scAxisExtra, with d_rr = isotropic d_r of d_r and d_zr = 1D d_z of
//      1D d_r, Sec. II.D) + rho g z^, and the hydrodynamic velocity
//      u = (j + F/2)/rho (Eq. uhydro) on a 2-node halo; halo rows outside the
//      domain take the mirrored velocity (u_z even, u_r odd at the axis, both
//      even at the wall);
//   4. per tile node: d_r u_z, d_z u_r, d_r u_r (isotropic stencil), the
//      source h_i (Eqs. condition_h, H_terms), u^eq = (j + tau F)/rho
//      (Eq. ueq), BGK collision (Eq. lbm2d_mod_new) and push-streaming into
//      the other buffer with the mid-grid specular axis, bounce-back or
//      specular wall and periodic z (Sec. II.E).
// HBM traffic per node and step: 9 population reads + 9 writes, plus the
// halo reloads that miss L2 (the side halos of neighbouring tiles mostly
// hit it; in all about 1.4x the 18 populations on 4096 x 512 in FP64).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

struct StepArgs {
    const void* fin;   // [9][nr][nz] storage type
    void* fout;        // [9][nr][nz] storage type (step mode)
    double* rho_out;   // moments mode, may be null
    double* uz_out;
    double* ur_out;
    double* partials;  // moments mode: [gridDim.x][4] block sums, may be null
    long long plane;   // population plane pitch in elements (>= nz * nr)
    unsigned state_bytes;  // 9 * plane * sizeof(storage) (< 4 GiB)
    int nz, nr;
    int tiles_z;       // tiles along z (tile id = tr * tiles_z + tz: z fastest)
    int big_nz;        // 1 if nz >= TZ + 6: periodic wrap needs one add/sub
    int reverse;       // 1: each XCD walks its run of tiles from the end
    int colmajor;      // 1: each XCD walks its run of whole tile rows column by column
    int wall;          // 0 no-slip, 1 free-slip
    int axisym;        // 1 axisymmetric terms on
    int opts;          // option bits: 1 Guo forcing, 2 no derivative terms across the wall,
                       // 4 no-slip walls at both ends of z, 8 open rows, 16 mid-link source
    double G, tau, rho0, gz, rho_ref;
    int in_row, out_row;    // open rows (option 8): inlet / outlet row, or -1
    double rho_bc_in, rho_bc_out;  // densities imposed there
    const double* u_in;      // [2][nz]: u_z then u_r imposed on the inlet row
    double* h_out;           // moments mode: [3][n] H_z, H_r, mass source of every node, may be null
    const double* h_in;      // option 16: the same fields, read at the far end of each link
};

// storage / compute precision of a kernel instance
template <class S_, class C_, bool kShift_>
struct Prec {
    using S = S_;
    using C = C_;
    static constexpr bool kShift = kShift_;  // storage holds f_i - W_i rho_ref
};
using PrecF64 = Prec<double, double, false>;
using PrecF32S = Prec<float, float, true>;

__device__ __forceinline__ double dev_exp(double x) { return exp(x); }
__device__ __forceinline__ float dev_exp(float x) { return expf(x); }

// 1/x from the hardware reciprocal refined by Newton steps (error well
// below 1e-15 relative in FP64), cheaper than an IEEE divide
__device__ __forceinline__ double dev_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float dev_rcp(float x) {
    float y = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(y, e, y);
}

// hardware dispatches workgroup b to XCD b % 8; renumber so that each XCD
// works on one contiguous run of tiles.  Tiles are numbered z fastest, so
// the workgroups resident on an XCD at one time cover whole rows of tiles
// and read each other's side halos through its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < rem ? x : rem) + k;
}

// the same runs, each walked from its last tile to its first
__device__ __forceinline__ int xcd_remap_rev(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7;
    const int x = b & 7, k = b >> 3;
    const int len = q + (x < rem ? 1 : 0);
    return x * q + (x < rem ? x : rem) + (len - 1 - k);
}

// the same runs, walked column by column (all the run's tile rows of one
// column, then the next column) when every run is a whole number of tile
// rows; otherwise as xcd_remap
__device__ __forceinline__ int xcd_remap_col(int b, int nb, int tiles_z) {
    const int q = nb >> 3, rem = nb & 7;
    if (rem != 0 || q % tiles_z != 0) return xcd_remap(b, nb);
    const int x = b & 7, k = b >> 3;
    const int rows = q / tiles_z;
    return x * q + (k % rows) * tiles_z + k / rows;
}

__device__ __forceinline__ int wrap_z(int z, int nz, bool big) {
    if (big) {
        z = z < 0 ? z + nz : z;
        return z >= nz ? z - nz : z;
    }
    int w = z % nz;
    return w < 0 ? w + nz : w;
}

// row of the node whose value a (possibly ghost) row takes: mirror about
// r = 0 below the axis and about r = nr above the wall; clamped into the
// array for rows no real node ever reads (partial tiles)
__device__ __forceinline__ int mirror_row(int y, int nr) {
    y = y < 0 ? -1 - y : y;
    y = y >= nr ? 2 * nr - 1 - y : y;
    y = y < 0 ? 0 : y;
    return y >= nr ? nr - 1 : y;
}

// position of window column x (>= 0) in an LDS row of W (even) entries: x
// itself, or (kSplit) the even columns first and the odd ones after them.
// With the split rows, lanes that hold z-adjacent node pairs (pair p at
// columns 2p, 2p + 1) read consecutive entries for any stencil offset, as
// lanes holding one node each do with plain rows.
template <bool kSplit>
__device__ __forceinline__ int lds_col(int x, int W) {
    return kSplit ? (x & 1) * (W >> 1) + (x >> 1) : x;
}

// isotropic first derivative (Sec. II.D): (1/36) sum_i (8 phi(x+c_i) -
// phi(x+2 c_i)) c_i,axis, on an LDS window of row pitch W
template <bool kAlongR, bool kSplit = false, class C>
__device__ __forceinline__ C d_iso(const C* __restrict__ E, int y, int x, int W) {
    C s = C(0);
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        const int c = kAlongR ? cr(i) : cz(i);
        if (c == 0) continue;
        const C t = C(8) * E[(y + cr(i)) * W + lds_col<kSplit>(x + cz(i), W)] -
                    E[(y + 2 * cr(i)) * W + lds_col<kSplit>(x + 2 * cz(i), W)];
        s += c > 0 ? t : -t;
    }
    return s * C(1.0 / 36.0);
}

// Populations are addressed through a buffer resource: the base and the
// plane offset i * plane * sizeof(S) are wave-uniform (scalar registers), the
// per-lane byte offset is 32-bit, so each load or store needs no vector
// address arithmetic.  Offsets beyond the buffer read as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// kAux: cache-policy bits of the store (16: device scope, written through
// the XCD's L2 to the memory-side cache)
template <int kAux = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, kAux);
}
template <int kAux = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, kAux);
}

// Two adjacent values in one access (16 bytes in FP64, 8 in FP32); the
// offset must be a multiple of the access size.  A 16-byte store takes its
// whole offset in the vector operand and 0 as the scalar one: a vector
// instruction that overwrites the data registers of a wider-than-8-byte
// buffer store right after it has corrupted the stored value on gfx950 also
// with a scalar-register offset, a form the compiler inserts no wait state
// for; with the constant offset it does.
typedef double pair_f64 __attribute__((ext_vector_type(2)));
typedef float pair_f32 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_load2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double& x,
                                          double& y) {
    const pair_f64 v = __builtin_bit_cast(pair_f64, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    x = v.x;
    y = v.y;
}
__device__ __forceinline__ void buf_load2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float& x,
                                          float& y) {
    const pair_f32 v = __builtin_bit_cast(pair_f32, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    x = v.x;
    y = v.y;
}
template <int kAux = 0>
__device__ __forceinline__ void buf_store2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double x,
                                           double y) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0u, 0u, 0));
    const pair_f64 v = {x, y};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, voff + soff, 0u, kAux);
}
template <int kAux = 0>
__device__ __forceinline__ void buf_store2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float x, float y) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    const pair_f32 v = {x, y};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, kAux);
}

// the value a lane one below (wave_shr:1) or one above (wave_shl:1) holds in
// the wave (DPP row/wave control codes of GFX9); the ends of the wave read 0
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
template <int kCtrl>
__device__ __forceinline__ double lane_from(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, kCtrl, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), kCtrl, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int kCtrl>
__device__ __forceinline__ float lane_from(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, 0xf, 0xf, false));
}

// One TZ x TR tile of one lattice: the whole step (or the moments) for the
// tile's nodes.  `tile` = tr * tiles_z + tz; `slot` indexes the per-block
// partial sums of the moments mode.  kOpt: the option bits, known at compile
// time (1: Guo forcing instead of the velocity shift; 2: the derivative terms
// -- F^{gamma,sym} and the velocity derivatives in H -- are zero on rows
// whose stencils reach across the outer wall), or -1: read at run time from
// StepArgs::opts (instances of a batch, and the two boundary options).
// Boundary options (Sec. II.E; run-time only): 4 closes both ends of z with
// mid-grid bounce-back walls at z = -1/2 and z = nz - 1/2 (psi is mirrored
// across them, the derivative terms whose stencils reach across are zero:
// F^{gamma,sym} on 4 columns, the velocity derivatives on 2 columns next to
// each wall); 8 imposes f^eq(rho_in, u_in(z)) on the inlet row and
// f^eq(rho_out, u one row inside) on the outlet row after the collision,
// with the derivative terms zero on rows whose stencils reach past them
// (F^{gamma,sym} within 3 rows inside, the velocity derivatives within 1,
// and every row outside).  Option 16 (run-time only): the source of each
// link is the average of h_i at its two ends, (h_i(x) + h_i(x + c_i)) / 2,
// with h_i(y) = W_i (mass(y) + 3 c_i . H(y)) from StepArgs::h_in (written by
// a moments pass with h_out); across the axis y is the mirror node with H_r
// reversed, across the outer wall the mirror node.  kStoreAux: cache-policy
// bits of the population stores (see buf_store).  kPair: a thread holds
// z-adjacent node pairs and, where nz and the plane pitch are even, z is
// periodic and the buffers aligned, moves each pair in one 16-byte (FP32: 8)
// access per plane, on LDS rows split into even and odd columns; the step is
// the same to the bit.  It is not the default: on 4096 x 512 it is slower
// (78.8 against 75.3 us per step in FP64): 13% more vector and 24% more LDS
// instructions and 2.5x the LDS bank conflicts outweigh 24% fewer memory
// reads.
template <class P, int TZ, int TR, int NT, bool kMoments, int kOpt = 0, int kStoreAux = 0, bool kPair = false>
__device__ __forceinline__ void tile_body(const StepArgs& a, const int tile, const int slot, const int t) {
    using S = typename P::S;
    using C = typename P::C;
    constexpr int PZ = TZ + 12, PR = TR + 12;  // psi window (halo 6)
    constexpr int DZ = TZ + 8, DR = TR + 8;    // d_r psi window (halo 4)
    constexpr int UZ = TZ + 4, UR = TR + 4;    // velocity window (halo 2)
    constexpr int NPT = TZ * TR / NT;          // tile nodes per thread
    static_assert(NPT * NT == TZ * TR, "tile must be a multiple of the workgroup");

    constexpr int NB = 4 * UZ;  // velocity ring: 2 rows below and 2 above the tile
    constexpr int NS = 4 * TR;  // and 2 columns left and 2 right
    constexpr int NU = NB + NS;

    __shared__ C s_psi[PR * PZ];
    __shared__ C s_dr[DR * DZ];
    __shared__ C s_d1[DR * DZ];  // 1D fourth-order d_r psi (rows 2 .. DR-3 used)
    __shared__ C s_uz[UR * UZ];
    __shared__ C s_ur[UR * UZ];
    __shared__ C s_mom[3][NU];  // rho, j_z, j_r of the velocity-ring nodes

    const __amdgpu_buffer_rsrc_t fin = pop_rsrc(a.fin, a.state_bytes);
    const unsigned plane_bytes = (unsigned)a.plane * (unsigned)sizeof(S);
    const int nz = a.nz, nr = a.nr;
    const bool big = a.big_nz != 0;
    const int tri = tile / a.tiles_z;
    const int z0 = (tile - tri * a.tiles_z) * TZ, r0 = tri * TR;
    const int opts = kOpt < 0 ? a.opts : kOpt;
    const bool guo = (opts & 1) != 0;
    const bool no_wall_deriv = (opts & 2) != 0;
    const bool zwalls = (opts & 4) != 0;
    const bool open = (opts & 8) != 0;
    const bool midlink = (opts & 16) != 0;
    const C rho0 = C(a.rho0);
    // column of the node a (possibly ghost) window column reads: periodic,
    // or mirrored about the z walls (clamped for columns no real node reads)
    auto col_of = [&](int z) {
        if (!zwalls) return wrap_z(z, nz, big);
        z = z < 0 ? -1 - z : z;
        z = z >= nz ? 2 * nz - 1 - z : z;
        z = z < 0 ? 0 : z;
        return z >= nz ? nz - 1 : z;
    };
    // F^{gamma,sym} and the velocity derivatives vanish where their
    // stencils would reach across a boundary other than the axis
    auto no_fsym = [&](int z, int r) {
        return (no_wall_deriv && r >= nr - 4) || (zwalls && (z < 4 || z >= nz - 4)) ||
               (open && ((a.in_row >= 0 && r <= a.in_row + 3) || (a.out_row >= 0 && r >= a.out_row - 3)));
    };
    auto no_du = [&](int z, int r) {
        return (no_wall_deriv && r >= nr - 2) || (zwalls && (z < 2 || z >= nz - 2)) ||
               (open && ((a.in_row >= 0 && r <= a.in_row + 1) || (a.out_row >= 0 && r >= a.out_row - 1)));
    };
    const C inv_rho0 = C(1.0 / a.rho0);
    const C rho_ref = C(a.rho_ref);

    auto psi_of = [&](C rho) { return rho0 * (C(1) - dev_exp(-rho * inv_rho0)); };

    auto rho_of = [&](const C* v) {
        C s = C(0);
#pragma unroll
        for (int i = 0; i < kQ; ++i) s += v[i];
        return P::kShift ? s + rho_ref : s;
    };
    auto jz_of = [](const C* v) { return (v[1] - v[3]) + (v[5] - v[6]) + (v[8] - v[7]); };
    auto jr_of = [](const C* v) { return (v[2] - v[4]) + (v[5] - v[8]) + (v[6] - v[7]); };

    // index of velocity-window node (uy, ux) in the compact ring arrays
    // (the node must lie outside the tile)
    auto ring_index = [](int uy, int ux) {
        if (uy < 2) return uy * UZ + ux;
        if (uy >= TR + 2) return (uy - TR) * UZ + ux;
        const int side = ux < 2 ? 0 : 1;
        return NB + side * 2 * TR + (uy - 2) * 2 + (side ? ux - TZ - 2 : ux);
    };

    // ---- 1. populations of the psi window (tile + 6-node ring) -----------
    // Every load is issued before any is used.  Ring nodes give psi and,
    // on the 2-node velocity ring, rho and j; tile nodes keep their
    // populations in registers until the collision.  Rows outside the
    // lattice read their mirror row (psi is even at the axis and the wall).
    constexpr int NBAND = 12 * PZ;  // 6 rows below and 6 above the tile
    constexpr int NSIDE = 12 * TR;  // 6 columns left and 6 right
    constexpr int NRING = NBAND + NSIDE;
    constexpr int NIT = (NRING + NT - 1) / NT;
    // a thread's tile nodes: one per row slot, or (kPair) z-adjacent pairs
    // (2p, 2p + 1) of a row, so that a pair moves in one access of both
    // values
    static_assert(!kPair || NPT % 2 == 0, "node pairs need an even count of nodes per thread");
    constexpr int ZL = kPair ? TZ / 2 : TZ;  // threads per tile row
    static_assert(NT % ZL == 0, "tile row must divide the workgroup");
    constexpr int RS = NT / ZL;  // rows between a thread's row slots
    const int lzb = kPair ? 2 * (t % ZL) : t % ZL, lrb = t / ZL;
    auto node_lz = [&](int k) { return kPair ? lzb + (k & 1) : lzb; };
    auto node_lr = [&](int k) { return kPair ? lrb + (k >> 1) * RS : lrb + k * RS; };
    // pair accesses need both nodes adjacent and the pair aligned to its
    // size in every plane: an even nz and pitch, aligned buffers and
    // periodic z (the mirror at z walls reverses a pair); (workgroup-uniform)
    const bool pio = kPair && ((nz & 1) | (a.plane & 1)) == 0 && !zwalls &&
                     ((reinterpret_cast<uintptr_t>(a.fin) | reinterpret_cast<uintptr_t>(a.fout)) &
                      (2 * sizeof(S) - 1)) == 0;
    // LDS windows: rows split into even and odd columns with node pairs
    auto lc = [](int x, int W) { return lds_col<kPair>(x, W); };
    C f[NPT][kQ];
    {
        C v[NIT][kQ];
        int hrz[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = t + it * NT;
            int hr, hz;
            if (idx < NBAND) {
                const int b = idx / PZ;
                hz = idx - b * PZ;
                hr = b < 6 ? b : TR + b;
            } else {
                const int j = idx - NBAND;
                const int side = j / (6 * TR);
                const int jj = j - side * 6 * TR;
                hr = 6 + jj / 6;
                hz = (side ? TZ + 6 : 0) + (jj - (jj / 6) * 6);
            }
            const bool live = idx < NRING;
            hrz[it] = live ? (hr << 16) | hz : -1;
            const int gz = col_of(z0 - 6 + hz);
            const int gr = mirror_row(r0 - 6 + (live ? hr : 6), nr);
            const unsigned node = (unsigned)(gr * nz + gz);
#pragma unroll
            for (int i = 0; i < kQ; ++i) v[it][i] = live ? C(buf_load(fin, node * (unsigned)sizeof(S), i * plane_bytes, S())) : C(0);
        }
        if (pio) {
#pragma unroll
            for (int k = 0; k < NPT; k += 2) {
                const unsigned node = (unsigned)(mirror_row(r0 + node_lr(k), nr) * nz + col_of(z0 + lzb));
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    S x, y;
                    buf_load2(fin, node * (unsigned)sizeof(S), i * plane_bytes, x, y);
                    f[k][i] = C(x);
                    f[k + 1][i] = C(y);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const unsigned node = (unsigned)(mirror_row(r0 + node_lr(k), nr) * nz + col_of(z0 + node_lz(k)));
#pragma unroll
                for (int i = 0; i < kQ; ++i)
                    f[k][i] = C(buf_load(fin, node * (unsigned)sizeof(S), i * plane_bytes, S()));
            }
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            if (hrz[it] < 0) continue;
            const int hr = hrz[it] >> 16, hz = hrz[it] & 0xffff;
            const C rho = rho_of(v[it]);
            s_psi[hr * PZ + lc(hz, PZ)] = psi_of(rho);
            const int uy = hr - 4, ux = hz - 4, gr = r0 - 6 + hr;
            if (uy >= 0 && uy < UR && ux >= 0 && ux < UZ && gr >= 0 && gr < nr) {
                const int o = ring_index(uy, ux);
                s_mom[0][o] = rho;
                s_mom[1][o] = jz_of(v[it]);
                s_mom[2][o] = jr_of(v[it]);
            }
        }
    }
    // the tile nodes' sums of the stored values (rho - rho_ref when shifted)
    // and j, formed once here and in 3a and read again by the collision
    C sig_t[NPT], jz_t[NPT], jr_t[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        C sg = C(0);
#pragma unroll
        for (int i = 0; i < kQ; ++i) sg += f[k][i];
        sig_t[k] = sg;
        s_psi[(node_lr(k) + 6) * PZ + lc(node_lz(k) + 6, PZ)] = psi_of(P::kShift ? sg + rho_ref : sg);
    }
    __syncthreads();

    // ---- 2. isotropic d_r psi on the 4-node halo, and the 1D d_r psi that
    // the mixed derivative d_zr differences along z ----------------------
    // (idx runs over LDS positions: with split rows, position q holds
    // column 2q, or 2 (q - DZ/2) + 1 in the row's second half)
    for (int idx = t; idx < DR * DZ; idx += NT) {
        const int y = idx / DZ, q = idx - y * DZ;
        const int x = kPair ? (q < DZ / 2 ? 2 * q : 2 * (q - DZ / 2) + 1) : q;
        s_dr[idx] = d_iso<true, kPair>(s_psi, y + 2, x + 2, PZ);
        if (y >= 2 && y < DR - 2) {
            const int c = lc(x + 2, PZ);  // psi-window column; rows y .. y + 4
            s_d1[idx] = (-s_psi[(y + 4) * PZ + c] + C(8) * s_psi[(y + 3) * PZ + c] - C(8) * s_psi[(y + 1) * PZ + c] +
                         s_psi[y * PZ + c]) *
                        C(1.0 / 12.0);
        }
    }
    __syncthreads();

    // ---- 3. total force and hydrodynamic velocity ------------------------
    const C G = C(a.G);
    const C g18 = G * C(1.0 / 18.0);  // (G/2) c_s^4
    const C gz_acc = C(a.gz);
    // force at velocity-window coordinates (uy, ux) of a real row whose
    // radius r + 1/2 has the reciprocal inv_r
    auto force_at = [&](int uy, int ux, C rho, C inv_r, C& Fz, C& Fr) {
        const int py = uy + 4, px = ux + 4;  // psi window
        const int dy = uy + 2, dx = ux + 2;  // d_r psi window
        C sz = C(0), sr = C(0);
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            const C ps = s_psi[(py + cr(i)) * PZ + lc(px + cz(i), PZ)] * C(weight(i));
            if (cz(i) != 0) sz += cz(i) > 0 ? ps : -ps;
            if (cr(i) != 0) sr += cr(i) > 0 ? ps : -ps;
        }
        const C psi = s_psi[py * PZ + lc(px, PZ)];
        Fz = -G * psi * sz;
        Fr = -G * psi * sr;
        // F^{gamma,sym} reads psi up to 4 rows away
        if (a.axisym && !no_fsym(z0 - 2 + ux, r0 - 2 + uy)) {
            const C dr1 = s_dr[dy * DZ + lc(dx, DZ)];
            const C drr = d_iso<true, kPair>(s_dr, dy, dx, DZ);
            // mixed derivative: 1D fourth-order d_z of the 1D fourth-order d_r
            const C* d1 = s_d1 + dy * DZ;
            const C dzr = (-d1[lc(dx + 2, DZ)] + C(8) * d1[lc(dx + 1, DZ)] - C(8) * d1[lc(dx - 1, DZ)] +
                           d1[lc(dx - 2, DZ)]) *
                          C(1.0 / 12.0);
            const C pre = -g18 * psi;
            Fz += pre * dzr * inv_r;
            Fr += pre * (drr * inv_r - dr1 * inv_r * inv_r);
        }
        Fz += rho * gz_acc;
    };

    C Fz_t[NPT], Fr_t[NPT];
    // 1 / (r + 1/2) and 1 / rho of the tile nodes, kept for the collision
    C inv_r_t[NPT], inv_rho_t[NPT];
    // 3a. tile nodes of real rows, from the populations in registers
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int lr = node_lr(k), lz = node_lz(k);
        const int gr = r0 + lr;
        Fz_t[k] = C(0);
        Fr_t[k] = C(0);
        inv_r_t[k] = C(0);
        inv_rho_t[k] = C(0);
        jz_t[k] = C(0);
        jr_t[k] = C(0);
        if (gr < nr) {
            const C rho = P::kShift ? sig_t[k] + rho_ref : sig_t[k];
            inv_r_t[k] = dev_rcp(C(gr) + C(0.5));
            C Fz, Fr;
            force_at(lr + 2, lz + 2, rho, inv_r_t[k], Fz, Fr);
            Fz_t[k] = Fz;
            Fr_t[k] = Fr;
            const C inv_rho = dev_rcp(rho);
            inv_rho_t[k] = inv_rho;
            jz_t[k] = jz_of(f[k]);
            jr_t[k] = jr_of(f[k]);
            s_uz[(lr + 2) * UZ + lc(lz + 2, UZ)] = (jz_t[k] + C(0.5) * Fz) * inv_rho;
            s_ur[(lr + 2) * UZ + lc(lz + 2, UZ)] = (jr_t[k] + C(0.5) * Fr) * inv_rho;
        }
    }
    // 3b. velocity-ring nodes of real rows, from rho and j in LDS
    for (int idx = t; idx < NU; idx += NT) {
        int uy, ux;
        if (idx < NB) {
            const int b = idx / UZ;
            ux = idx - b * UZ;
            uy = b < 2 ? b : TR + b;
        } else {
            const int j = idx - NB;
            const int side = j / (2 * TR);
            const int jj = j - side * 2 * TR;
            uy = 2 + (jj >> 1);
            ux = (side ? TZ + 2 : 0) + (jj & 1);
        }
        const int y = r0 - 2 + uy;
        if (y < 0 || y >= nr) continue;
        const C rho = s_mom[0][idx];
        C Fz, Fr;
        force_at(uy, ux, rho, dev_rcp(C(y) + C(0.5)), Fz, Fr);
        const C inv_rho = dev_rcp(rho);
        s_uz[uy * UZ + lc(ux, UZ)] = (s_mom[1][idx] + C(0.5) * Fz) * inv_rho;
        s_ur[uy * UZ + lc(ux, UZ)] = (s_mom[2][idx] + C(0.5) * Fr) * inv_rho;
    }
    __syncthreads();
    // 3c. rows outside the lattice (only in tiles at the axis or the wall):
    // the velocity of the mirror row, u_r odd at the axis and even at the
    // wall; entries no real node reads are zeroed
    const int axis_rows = r0 < 2 ? 2 - r0 : 0;  // velocity-window rows below the axis
    const int wall_lo = nr - (r0 - 2);           // first velocity-window row beyond the wall
    if (axis_rows > 0 || wall_lo < UR) {         // uniform over the workgroup
        // (a copy within one LDS column position: the same column in
        // either row layout)
        for (int idx = t; idx < UR * UZ; idx += NT) {
            const int uy = idx / UZ, ux = idx - uy * UZ;
            const bool axis_side = uy < axis_rows;
            if (!axis_side && uy < wall_lo) continue;
            const int y = r0 - 2 + uy;
            const int ys = axis_side ? -1 - y : 2 * nr - 1 - y;
            const C sgn = axis_side ? C(-1) : C(1);
            const int uys = ys - (r0 - 2);
            if (ys < 0 || ys >= nr || uys < 0 || uys >= UR) {
                s_uz[idx] = C(0);
                s_ur[idx] = C(0);
            } else {
                s_uz[idx] = s_uz[uys * UZ + ux];
                s_ur[idx] = sgn * s_ur[uys * UZ + ux];
            }
        }
        __syncthreads();
    }

    // ---- 4. collision + streaming (or moments) for the tile nodes --------
    // (uniform over the workgroup) no tile row is the axis row or the wall
    // row, no push crosses the ends of z, and no z walls
    const bool plain = !zwalls && r0 >= 1 && r0 + TR <= nr - 1 && z0 >= 1 && z0 + TZ <= nz - 1;
    const C tau = C(a.tau);
    const C inv_tau = C(1) / tau;
    const C mu_fac = (tau - C(0.5)) * C(1.0 / 3.0);  // mu = rho c_s^2 (tau - 1/2)
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    // push of an interior pair (nodes 2p, 2p + 1 of a tile row at byte
    // offset a_off) in aligned pairs: the pushes along r land on the pair's
    // own columns; along +z the target pair (2p, 2p + 1) takes the second
    // node of pair p - 1 (one lane below) and this pair's first node, along
    // -z this pair's second node and the first node of pair p + 1 (one lane
    // above).  The ends of a tile row store their odd value alone.
    auto push_pair = [&](unsigned a_off, const C* fa, const C* fb) {
        const __amdgpu_buffer_rsrc_t fo = pop_rsrc(a.fout, a.state_bytes);
        const int p = t % ZL;
        const bool first = p == 0, last = p == ZL - 1;
        constexpr unsigned sz = (unsigned)sizeof(S);
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const unsigned soff = (unsigned)i * plane_bytes + (unsigned)(cr(i) * nz * (int)sizeof(S));
            const S va = S(fa[i]), vb = S(fb[i]);
            if (cz(i) == 0) {
                buf_store2<kStoreAux>(fo, a_off, soff, va, vb);
            } else if (cz(i) > 0) {
                const S prev_b = lane_from<kDppWaveShr1>(vb);
                if (!first) buf_store2<kStoreAux>(fo, a_off, soff, prev_b, va);
                else buf_store<kStoreAux>(fo, a_off + sz, soff, va);
                if (last) buf_store<kStoreAux>(fo, a_off + 2 * sz, soff, vb);
            } else {
                const S next_a = lane_from<kDppWaveShl1>(va);
                if (!last) buf_store2<kStoreAux>(fo, a_off, soff, vb, next_a);
                else buf_store<kStoreAux>(fo, a_off, soff, vb);
                if (first) buf_store<kStoreAux>(fo, a_off - sz, soff, va);
            }
        }
    };
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int lr = node_lr(k), lz = node_lz(k);
        const int gz = z0 + lz, gr = r0 + lr;
        const bool valid = gz < nz && gr < nr;
        if (!valid) continue;
        const int uy = lr + 2, ux = lz + 2;
        const C sig = sig_t[k];  // sum of the stored values: rho - rho_ref when shifted
        const C rho = P::kShift ? sig + rho_ref : sig;
        const C jz = jz_t[k], jr = jr_t[k];
        const C uz = s_uz[uy * UZ + lc(ux, UZ)], ur = s_ur[uy * UZ + lc(ux, UZ)];
        const C rr = C(gr) + C(0.5);

        // H and the mass source of the node (Eqs. H_terms, condition_h)
        auto source_terms = [&](C& hz, C& hr, C& mass) {
            // the velocity derivatives read rows up to 2 away
            const bool zd = no_du(gz, gr);
            const C druz = zd ? C(0) : d_iso<true, kPair>(s_uz, uy, ux, UZ);
            const C dzur = zd ? C(0) : d_iso<false, kPair>(s_ur, uy, ux, UZ);
            const C drur = zd ? C(0) : d_iso<true, kPair>(s_ur, uy, ux, UZ);
            const C inv_r = inv_r_t[k];
            const C mu = rho * mu_fac;
            hz = (mu * (druz + dzur) - rho * ur * uz) * inv_r;
            hr = (C(2) * mu * (drur - ur * inv_r) - rho * ur * ur) * inv_r;
            mass = -rho * ur * inv_r;
        };

        if constexpr (kMoments) {
            // the moments and the global sums are formed in FP64 from the
            // stored values (in FP32 storage the nine values and rho_ref are
            // added in double; the force stays that of the FP32 step)
            double rho_d = 0.0;
#pragma unroll
            for (int i = 0; i < kQ; ++i) rho_d += double(f[k][i]);
            if (P::kShift) rho_d += a.rho_ref;
            auto dv = [&](int i) { return double(f[k][i]); };
            const double jz_d = (dv(1) - dv(3)) + (dv(5) - dv(6)) + (dv(8) - dv(7));
            const double jr_d = (dv(2) - dv(4)) + (dv(5) - dv(8)) + (dv(6) - dv(7));
            const double inv_rho_d = dev_rcp(rho_d);
            const double uz_d = (jz_d + 0.5 * double(Fz_t[k])) * inv_rho_d;
            const double ur_d = (jr_d + 0.5 * double(Fr_t[k])) * inv_rho_d;
            const long long x = (long long)gr * nz + gz;
            if (a.rho_out) a.rho_out[x] = rho_d;
            if (a.uz_out) a.uz_out[x] = uz_d;
            if (a.ur_out) a.ur_out[x] = ur_d;
            if (a.h_out) {
                C hz = C(0), hr = C(0), mass = C(0);
                if (a.axisym) source_terms(hz, hr, mass);
                const long long hn = (long long)nz * nr;  // the H fields are [3][nr][nz]
                a.h_out[x] = double(hz);
                a.h_out[hn + x] = double(hr);
                a.h_out[2 * hn + x] = double(mass);
            }
            const double two_pi_r = 6.283185307179586 * double(rr);
            part[0] += two_pi_r * rho_d;
            part[1] += two_pi_r * rho_d * uz_d;
            part[2] += 0.5 * two_pi_r * rho_d * (uz_d * uz_d + ur_d * ur_d);
            part[3] += rho_d;
        } else {
            const C Fz = Fz_t[k], Fr = Fr_t[k];
            C hz = C(0), hr = C(0), mass = C(0);
            if (a.axisym) source_terms(hz, hr, mass);
            const C inv_rho = inv_rho_t[k];  // rho is summed as in 3a
            // equilibrium velocity: shifted by tau F (Eq. ueq), or the
            // hydrodynamic velocity with Guo forcing
            const C qz = guo ? uz : (jz + tau * Fz) * inv_rho;
            const C qr = guo ? ur : (jr + tau * Fr) * inv_rho;
            const C qq = C(1.5) * (qz * qz + qr * qr);
            const C gpre = C(1) - C(0.5) * inv_tau;  // Guo: (1 - 1/(2 tau))
            const C uF = uz * Fz + ur * Fr;
            // open rows: the imposed equilibrium replaces the collision
            const bool bc = open && (gr == a.in_row || gr == a.out_row);
            C brho = C(0), bz = C(0), br = C(0);
            if (bc) {
                if (gr == a.in_row) {
                    brho = C(a.rho_bc_in);
                    bz = C(a.u_in[gz]);
                    br = C(a.u_in[nz + gz]);
                } else {
                    brho = C(a.rho_bc_out);
                    bz = s_uz[(uy - 1) * UZ + lc(ux, UZ)];
                    br = s_ur[(uy - 1) * UZ + lc(ux, UZ)];
                }
            }
            const C bqq = C(1.5) * (bz * bz + br * br);
            const __amdgpu_buffer_rsrc_t fout = pop_rsrc(a.fout, a.state_bytes);
            // FP32 weights sum to 1 + 7.45e-9, which would bias the mass of
            // f^eq (and of h) by that fraction at every collision; in FP32 the
            // rest direction is therefore taken last, as the remainder that
            // makes sum_i f^eq_i = rho and sum_i h_i = -rho u_r / r hold
            // (both hold exactly for the paper's weights)
            constexpr bool kRem = sizeof(C) == 4;
            C feq_acc = C(0), h_acc = C(0);
#pragma unroll
            for (int ii = 0; ii < kQ; ++ii) {
                const int i = kRem ? (ii + 1) % kQ : ii;
                const C w = C(weight(i));
                C feq, hi, hsrc = C(0);
                if (kRem && i == 0) {
                    // the Guo term carries no mass either: its rest part is
                    // minus the sum of the others
                    feq = sig - feq_acc;
                    hi = mass - h_acc;
                } else {
                    const C cu = C(cz(i)) * qz + C(cr(i)) * qr;
                    const C poly = C(3) * cu + C(4.5) * cu * cu - qq;
                    // f^eq(rho, u^eq) (Eq. e_distribution with u^eq
                    // throughout); in shifted storage, f^eq - W rho_ref
                    feq = P::kShift ? w * (sig + rho * poly) : w * rho * (C(1) + poly);
                    hsrc = w * (mass + C(3) * (C(cz(i)) * hz + C(cr(i)) * hr));
                    hi = hsrc;
                    if (guo) {
                        // Guo et al.: W_i [3 (c_i - u) + 9 (c_i . u) c_i] . F
                        const C cF = C(cz(i)) * Fz + C(cr(i)) * Fr;
                        const C cuu = C(cz(i)) * uz + C(cr(i)) * ur;
                        hi += gpre * w * (C(3) * (cF - uF) + C(9) * cuu * cF);
                    }
                    feq_acc += feq;
                    h_acc += hi;
                }
                if (midlink && i != 0) {
                    // the source at the far end of the link, from that node's fields
                    int yr = gr + cr(i);
                    C sr = C(1);  // H_r is odd across the axis
                    if (yr < 0) {
                        yr = -1 - yr;
                        sr = C(-1);
                    } else if (yr >= nr) {
                        yr = 2 * nr - 1 - yr;
                    }
                    int yz = gz + cz(i);
                    yz = yz < 0 ? yz + nz : (yz >= nz ? yz - nz : yz);
                    const long long y = (long long)yr * nz + yz;
                    const long long hn = (long long)nz * nr;
                    const C hy = w * (C(a.h_in[2 * hn + y]) +
                                      C(3) * (C(cz(i)) * C(a.h_in[y]) + C(cr(i)) * sr * C(a.h_in[hn + y])));
                    hi += C(0.5) * (hy - hsrc);  // the source part only: (h_i(x) + h_i(y)) / 2
                }
                C fs = f[k][i] - (f[k][i] - feq) * inv_tau + hi;
                if (bc) {
                    const C cb = C(cz(i)) * bz + C(cr(i)) * br;
                    const C e = w * brho * (C(1) + C(3) * cb + C(4.5) * cb * cb - bqq);
                    fs = P::kShift ? e - w * rho_ref : e;
                }
                f[k][i] = fs;  // the pre-collision value is not read again
            }
            // push to the neighbours with the pre-streaming boundary rules.
            // A tile that holds neither the axis row nor the wall row and
            // needs no wrap in z sends population i to (z + c_z, r + c_r)
            // in plane i: one vector offset for all nine stores, the
            // displacement folded into the scalar offset.
            if (plain) {
                const unsigned node_off = (unsigned)(gr * nz + gz) * (unsigned)sizeof(S);
                if (kPair && pio) {
                    // a pair is pushed once its second node is done (both lie
                    // in one row and are valid: nz is even)
                    if (k & 1) push_pair(node_off - (unsigned)sizeof(S), f[k - 1], f[k]);
                } else {
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        // i * plane + displacement is the (non-negative) offset of the
                        // target in plane i; unsigned wrap-around adds the signed
                        // displacement exactly
                        const unsigned disp = (unsigned)((cr(i) * nz + cz(i)) * (int)sizeof(S));
                        buf_store<kStoreAux>(fout, node_off, (unsigned)i * plane_bytes + disp, S(f[k][i]));
                    }
                }
            } else if (!zwalls && gr > 0 && gr < nr - 1) {
                // a row between the axis and the wall in a tile at an end of
                // z (or on a lattice narrower than a tile): the same push, the
                // targets across a periodic end moved by one period
                const unsigned node_off = (unsigned)(gr * nz + gz) * (unsigned)sizeof(S);
                const unsigned period = (unsigned)nz * (unsigned)sizeof(S);
                const unsigned off_m = gz == 0 ? node_off + period : node_off;       // c_z = -1
                const unsigned off_p = gz == nz - 1 ? node_off - period : node_off;  // c_z = +1 (gr >= 1)
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const unsigned disp = (unsigned)((cr(i) * nz + cz(i)) * (int)sizeof(S));
                    buf_store<kStoreAux>(fout, cz(i) < 0 ? off_m : (cz(i) > 0 ? off_p : node_off),
                                         (unsigned)i * plane_bytes + disp, S(f[k][i]));
                }
            } else {
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    int tz = gz + cz(i), trr = gr + cr(i), d = i;
                    if (zwalls && (tz < 0 || tz >= nz)) {
                        // a z wall: the population returns to its node reversed
                        tz = gz;
                        trr = gr;
                        d = opposite(i);
                    } else if (cr(i) < 0 && gr == 0) {
                        trr = 0;
                        d = mirror_r(i);
                    } else if (cr(i) > 0 && gr == nr - 1) {
                        if (a.wall == 0) {
                            tz = gz;
                            trr = gr;
                            d = opposite(i);
                        } else {
                            d = mirror_r(i);
                            trr = gr;
                        }
                    }
                    tz = tz < 0 ? tz + nz : (tz >= nz ? tz - nz : tz);
                    buf_store<kStoreAux>(fout, (unsigned)(trr * nz + tz) * (unsigned)sizeof(S), d * plane_bytes,
                                         S(f[k][i]));
                }
            }
        }
    }

    if constexpr (kMoments) {
        if (a.partials) {
            __shared__ double s_red[4][NT / 64];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                double v = part[m];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
                if ((t & 63) == 0) s_red[m][t >> 6] = v;
            }
            __syncthreads();
            if (t < 4) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) v += s_red[t][w];
                a.partials[(long long)slot * 4 + t] = v;
            }
        }
    }
}

// tile of workgroup b (nb workgroups, one per tile) in slab order: XCD b % 8
// takes a slab of tiles_z / 8 tile columns (when 8 divides tiles_z; else the
// contiguous run of whole tile rows of xcd_remap) and walks it z fastest, so
// the workgroups resident on an XCD form a compact block of tiles and each
// round of tiles sits just above the previous one.
__device__ __forceinline__ int slab_tile(int b, int nb, int tiles_z) {
    if ((tiles_z & 7) != 0) return xcd_remap(b, nb);
    const int sw = tiles_z >> 3, k = b >> 3;
    const int tr = k / sw;
    return tr * tiles_z + (b & 7) * sw + (k - tr * sw);
}

// kSlab: slab order (slab_tile) instead of runs of tile rows (xcd_remap);
// kPair: each thread holds z-adjacent node pairs (see tile_body)
template <class P, int TZ, int TR, int NT, bool kMoments, int kOpt = 0, bool kSlab = false, int kStoreAux = 0,
          bool kPair = false>
__global__ __launch_bounds__(NT) void axi_tile_kernel(const StepArgs a) {
    const int tile = kSlab ? slab_tile(blockIdx.x, gridDim.x, a.tiles_z)
                           : (a.colmajor ? xcd_remap_col(blockIdx.x, gridDim.x, a.tiles_z)
                                         : (a.reverse ? xcd_remap_rev(blockIdx.x, gridDim.x)
                                                      : xcd_remap(blockIdx.x, gridDim.x)));
    tile_body<P, TZ, TR, NT, kMoments, kOpt, kStoreAux, kPair>(a, tile, blockIdx.x, threadIdx.x);
}

}  // namespace lbm
