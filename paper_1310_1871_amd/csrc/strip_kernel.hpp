// Row-marching form of the fused step of the axisymmetric Shan–Chen lattice
// Boltzmann method (Srivastava et al., arXiv:1310.1871, Sec. II): the same
// arithmetic as tile_body (step_kernel.hpp), organised so that no halo row is
// read or recomputed twice.
//
// A workgroup owns a band of 64 columns (z) and a chunk of rows (r).  It walks
// up the chunk in slabs of 4 rows.  Each iteration reads the populations of
// the 4 rows that lie 6 rows above the slab (the look-ahead the psi stencils
// need: F^{gamma,sym} at the velocity ring, 2 rows around a node, takes d_rr =
// d_r d_r psi, 2 + 2 + 2 rows), plus 6 columns on each side of the band, and
// forms psi(rho), rho and j for them (Sec. II.A).  The isotropic d_r psi (Sec. II.D),
// the 1D d_r psi of the mixed derivative, the force F = F^SC (Eq. scforce) +
// F^{gamma,sym} (Eq. scAxisExtra) + rho g z^ and the hydrodynamic velocity u
// (Eq. uhydro) then follow for the rows that have become computable, and the
// slab itself is collided (Eqs. condition_h, H_terms, ueq, lbm2d_mod_new)
// and pushed into the other buffer with the boundary links of Sec. II.E.
//
// psi (16 rows), d_r psi, rho, j and u (8 rows) live in circular LDS windows
// (row l in slot l mod rows).  The populations of a row are read for psi, rho and j,
// and read again one iteration later for the collision (from L2, where the
// first read left them: keeping them in registers for that iteration would
// double the registers and halve the workgroups per compute unit).  Per
// node and step the band reads 76/64 of its populations from memory (the
// side columns, which the neighbouring bands read at about the same time,
// mostly from L2), plus 12 rows per chunk; it computes psi for 76/64, d_r psi
// for 72/64 and the force for 68/64 of its nodes, against 2.1, 1.7 and 1.3
// for a 64 x 16 tile with a 6-node ring.
//
// Rows outside the lattice take the value of their mirror row (psi even at
// the axis and at the wall; u_z even and u_r odd at the axis, both even at
// the wall: the derivative rule of Sec. II.E), columns wrap periodically.
// Options: kOpt bit 1 Guo forcing, bit 2 no derivative terms across the wall
// (the readings of tile_body); the other options go through tile_body.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "step_kernel.hpp"

namespace lbm {

struct StripArgs {
    int chunk_rows;  // rows per chunk, a multiple of the slab height
    int chunks;      // chunks per band (ceil(nr / chunk_rows))
};

constexpr int kStripW = 64;   // band width (columns)
constexpr int kStripS = 4;    // slab height (rows): one wave per SIMD
constexpr int kStripNT = kStripW * kStripS;

template <class P, int kOpt, int kStoreAux>
__global__ __launch_bounds__(kStripNT) void axi_strip_kernel(const StepArgs a, const StripArgs sa) {
    using S = typename P::S;
    using C = typename P::C;
    constexpr int W = kStripW, SR = kStripS, NT = kStripNT;
    constexpr int PW = W + 12, DW = W + 8, UW = W + 4;  // window widths: psi, d_r psi, u
    // rows per circular window: psi holds rows [S k - 6, S k + S + 6) at the
    // start of the loop and [S k, S k + S + 6) in it; d_r psi [S k, S k + S + 4);
    // u [S k - 2, S k + S + 2); rho and j [S k + 2, S k + S + 6)
    constexpr int NP = 16, NW = 8;
    static_assert(SR + 6 <= NP && 12 <= NP && SR + 4 <= NW && 8 <= NW, "windows too short");
    constexpr int NSIDE = 12 * SR;                        // side nodes of a slab of fresh rows
    static_assert(NSIDE <= NT && 4 * SR <= NT && SR >= 2, "side work must fit the workgroup");
    constexpr int KPRO = (12 + SR - 1) / SR;              // iterations that fill the windows first

    __shared__ C s_psi[NP * PW];
    __shared__ C s_dr[NW * DW];
    __shared__ C s_d1[SR * DW];          // 1D d_r psi of the rows whose force is due
    __shared__ C s_uz[NW * UW];
    __shared__ C s_ur[NW * UW];
    __shared__ C s_mj[3][NW * UW];       // rho, j_z, j_r on the u window

    const int nz = a.nz, nr = a.nr;
    const bool big = a.big_nz != 0;
    const int id = xcd_remap(blockIdx.x, gridDim.x);  // each XCD: a run of whole bands
    const int band = id / sa.chunks;
    const int chunk = id - band * sa.chunks;
    const int c0 = band * W;
    const int R0 = chunk * sa.chunk_rows;
    const int R1 = min(nr, R0 + sa.chunk_rows);
    const int t = threadIdx.x;
    const int lz = t & (W - 1), lr = t / W;
    // side node of a thread t < NSIDE: row sr of the fresh rows, psi-window
    // column swx (0..5 left of the band, W+6..W+11 right of it)
    const int sr = t / 12, sc = t - (t / 12) * 12;
    const int swx = sc < 6 ? sc : W + sc;

    const __amdgpu_buffer_rsrc_t fin = pop_rsrc(a.fin, a.state_bytes);
    const __amdgpu_buffer_rsrc_t fout = pop_rsrc(a.fout, a.state_bytes);
    const unsigned plane_bytes = (unsigned)a.plane * (unsigned)sizeof(S);
    const int opts = kOpt;
    const bool guo = (opts & 1) != 0;
    const bool no_wall_deriv = (opts & 2) != 0;
    const C rho0 = C(a.rho0);
    const C inv_rho0 = C(1.0 / a.rho0);
    const C rho_ref = C(a.rho_ref);

    auto slot = [](int l) { return l & (NP - 1); };   // psi window
    auto wslot = [](int l) { return l & (NW - 1); };  // the other windows
    auto psi_of = [&](C rho) { return rho0 * (C(1) - dev_exp(-rho * inv_rho0)); };
    auto rho_of = [&](const C* v) {
        C s = C(0);
#pragma unroll
        for (int i = 0; i < kQ; ++i) s += v[i];
        return P::kShift ? s + rho_ref : s;
    };
    auto jz_of = [](const C* v) { return (v[1] - v[3]) + (v[5] - v[6]) + (v[8] - v[7]); };
    auto jr_of = [](const C* v) { return (v[2] - v[4]) + (v[5] - v[8]) + (v[6] - v[7]); };
    auto load9 = [&](int l, int wz, C* v) {
        const int gr = mirror_row(R0 + l, nr);
        const int gz = wrap_z(c0 + wz, nz, big);
        const unsigned off = (unsigned)(gr * nz + gz) * (unsigned)sizeof(S);
#pragma unroll
        for (int i = 0; i < kQ; ++i) v[i] = C(buf_load(fin, off, i * plane_bytes, S()));
    };
    // isotropic first derivative along r (Sec. II.D) of a circular window of
    // row pitch PITCH at local row l, window column x; the terms are summed
    // in the order of d_iso
    auto d_r_win = [&](const C* E, int pitch, int mask, int l, int x) {
        C s = C(0);
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            const int c = cr(i);
            if (c == 0) continue;
            const C tt = C(8) * E[((l + cr(i)) & mask) * pitch + x + cz(i)] -
                         E[((l + 2 * cr(i)) & mask) * pitch + x + 2 * cz(i)];
            s += c > 0 ? tt : -tt;
        }
        return s * C(1.0 / 36.0);
    };
    auto d_z_win = [&](const C* E, int pitch, int mask, int l, int x) {
        C s = C(0);
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            const int c = cz(i);
            if (c == 0) continue;
            const C tt = C(8) * E[((l + cr(i)) & mask) * pitch + x + cz(i)] -
                         E[((l + 2 * cr(i)) & mask) * pitch + x + 2 * cz(i)];
            s += c > 0 ? tt : -tt;
        }
        return s * C(1.0 / 36.0);
    };

    const C G = C(a.G);
    const C g18 = G * C(1.0 / 18.0);  // (G/2) c_s^4
    const C gz_acc = C(a.gz);
    // total force at local row l (global row gr), u-window column ux; d1row:
    // row of s_d1 holding this row's 1D d_r psi
    auto force_at = [&](int l, int gr, int ux, int d1row, C rho, C& Fz, C& Fr) {
        const int px = ux + 4, dx = ux + 2;
        C sz = C(0), srr = C(0);
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            const C ps = s_psi[slot(l + cr(i)) * PW + px + cz(i)] * C(weight(i));
            if (cz(i) != 0) sz += cz(i) > 0 ? ps : -ps;
            if (cr(i) != 0) srr += cr(i) > 0 ? ps : -ps;
        }
        const C psi = s_psi[slot(l) * PW + px];
        Fz = -G * psi * sz;
        Fr = -G * psi * srr;
        if (a.axisym && !(no_wall_deriv && gr >= nr - 4)) {
            const C dr1 = s_dr[wslot(l) * DW + dx];
            const C drr = d_r_win(s_dr, DW, NW - 1, l, dx);
            const C* d1 = s_d1 + d1row * DW + dx - 2;
            const C dzr = (-d1[4] + C(8) * d1[3] - C(8) * d1[1] + d1[0]) * C(1.0 / 12.0);
            const C inv_r = dev_rcp(C(gr) + C(0.5));
            const C pre = -g18 * psi;
            Fz += pre * dzr * inv_r;
            Fr += pre * (drr * inv_r - dr1 * inv_r * inv_r);
        }
        Fz += rho * gz_acc;
    };

    const C tau = C(a.tau);
    const C inv_tau = C(1) / tau;
    const C mu_fac = (tau - C(0.5)) * C(1.0 / 3.0);  // mu = rho c_s^2 (tau - 1/2)
    const bool band_inner = c0 >= 1 && c0 + W <= nz - 1;

    C fc[kQ], ff[kQ];                 // populations: the slab node (collision), the fresh node
    C Fzc = C(0), Frc = C(0);         // force at the slab node
    C Fzn = C(0), Frn = C(0);         // force at the fresh node (rows lr < 2)
    const int K = (R1 - R0 + SR - 1) / SR;  // slabs of the chunk

    // Iteration k collides local rows [SR k, SR k + SR) (global row = R0 +
    // local row).  k = -KPRO .. -1 fill the windows below the first slab.
    for (int k = -KPRO; k < K; ++k) {
        const int F0 = SR * k + 6;  // first fresh local row: 6 rows above the slab start
        // ---- A. populations of the fresh rows (every load before any use)
        load9(F0 + lr, lz, ff);
        C sv[kQ];
        const bool side = t < NSIDE;
        if (side) load9(F0 + sr, swx - 6, sv);
        // ---- B. psi of the fresh rows, and rho, j on the u window
        {
            const C rho = rho_of(ff);
            s_psi[slot(F0 + lr) * PW + lz + 6] = psi_of(rho);
            const int q = wslot(F0 + lr) * UW + lz + 2;
            s_mj[0][q] = rho;
            s_mj[1][q] = jz_of(ff);
            s_mj[2][q] = jr_of(ff);
        }
        if (side) {
            const C rho = rho_of(sv);
            s_psi[slot(F0 + sr) * PW + swx] = psi_of(rho);
            if (sc >= 4 && sc < 8) {
                const int q = wslot(F0 + sr) * UW + (sc < 6 ? sc - 4 : W + sc - 4);
                s_mj[0][q] = rho;
                s_mj[1][q] = jz_of(sv);
                s_mj[2][q] = jr_of(sv);
            }
        }
        __syncthreads();
        if (k < -1) continue;

        // ---- C. d_r psi for the rows 4 .. S+3 above the slab start (and
        // from 4 below it before the first slab), 1D d_r psi for the rows
        // 2 .. S+1
        {
            const int dlo = k < 0 ? -4 : SR * k + 4;
            const int dn = (k < 0 ? SR + 4 : SR) * DW;
            for (int idx = t; idx < dn; idx += NT) {
                const int y = idx / DW, x = idx - (idx / DW) * DW;
                s_dr[wslot(dlo + y) * DW + x] = d_r_win(s_psi, PW, NP - 1, dlo + y, x + 2);
            }
            const int l1 = SR * k + 2;
            for (int idx = t; idx < SR * DW; idx += NT) {
                const int y = idx / DW, x = idx - (idx / DW) * DW;
                const int l = l1 + y, c = x + 2;
                s_d1[idx] = (-s_psi[slot(l + 2) * PW + c] + C(8) * s_psi[slot(l + 1) * PW + c] -
                             C(8) * s_psi[slot(l - 1) * PW + c] + s_psi[slot(l - 2) * PW + c]) *
                            C(1.0 / 12.0);
            }
        }
        __syncthreads();

        // ---- D. force and hydrodynamic velocity of the rows 2 .. S+1 above
        // the slab start, from rho and j on the u window.  The populations
        // of the slab, read one iteration ago, are read again for the
        // collision (they are still in L2)
        const int lc = SR * k + lr;  // local row of this thread's slab node
        const int gcr = R0 + lc, gcz = c0 + lz;
        const bool coll = k >= 0 && gcr < R1 && gcz < nz;
        if (coll) {
            const unsigned off = (unsigned)(gcr * nz + gcz) * (unsigned)sizeof(S);
#pragma unroll
            for (int i = 0; i < kQ; ++i) fc[i] = C(buf_load(fin, off, i * plane_bytes, S()));
        }
        {
            const int lF = lr >= 2 ? SR * k + lr : SR * k + SR + lr;
            const int g = R0 + lF;
            const bool need = (k >= 0 || lF >= -2) && g >= 0 && g < nr;
            if (need) {
                const int q = wslot(lF) * UW + lz + 2;
                const C rho = s_mj[0][q];
                C Fz, Fr;
                force_at(lF, g, lz + 2, lF - (SR * k + 2), rho, Fz, Fr);
                const C inv_rho = dev_rcp(rho);
                s_uz[q] = (s_mj[1][q] + C(0.5) * Fz) * inv_rho;
                s_ur[q] = (s_mj[2][q] + C(0.5) * Fr) * inv_rho;
                if (lr >= 2) {
                    Fzc = Fz;
                    Frc = Fr;
                } else {
                    Fzn = Fz;
                    Frn = Fr;
                }
            }
            if (t < 4 * SR) {
                const int y = t >> 2, qq = t & 3;
                const int l = SR * k + 2 + y;
                const int gs = R0 + l;
                if ((k >= 0 || l >= -2) && gs >= 0 && gs < nr) {
                    const int ux = qq < 2 ? qq : W + qq;  // u-window columns 0, 1, W+2, W+3
                    const int m = wslot(l) * UW + ux;
                    const C rho = s_mj[0][m];
                    C Fz, Fr;
                    force_at(l, gs, ux, y, rho, Fz, Fr);
                    const C inv_rho = dev_rcp(rho);
                    s_uz[m] = (s_mj[1][m] + C(0.5) * Fz) * inv_rho;
                    s_ur[m] = (s_mj[2][m] + C(0.5) * Fr) * inv_rho;
                }
            }
        }
        __syncthreads();
        // rows just outside the lattice among the rows computed above: the
        // velocity of the mirror row (u_r odd at the axis, even at the wall)
        {
            const int ulo = k < 0 ? -2 : SR * k + 2, uhi = SR * k + SR + 2;
            const int glo = R0 + ulo, ghi = R0 + uhi;
            if (glo < 0 || ghi > nr) {  // uniform over the workgroup
                for (int idx = t; idx < (uhi - ulo) * UW; idx += NT) {
                    const int y = idx / UW, x = idx - (idx / UW) * UW;
                    const int l = ulo + y, g = R0 + l;
                    if (!((g >= -2 && g < 0) || (g >= nr && g < nr + 2))) continue;
                    const bool axis_side = g < 0;
                    const int ls = (axis_side ? -1 - g : 2 * nr - 1 - g) - R0;
                    s_uz[wslot(l) * UW + x] = s_uz[wslot(ls) * UW + x];
                    s_ur[wslot(l) * UW + x] = (axis_side ? C(-1) : C(1)) * s_ur[wslot(ls) * UW + x];
                }
                __syncthreads();
            }
        }
        if (k < 0) {
            if (lr < 2) {
                Fzc = Fzn;
                Frc = Frn;
            }
            continue;
        }

        // ---- E. collision and push of the slab
        {
            const int l = lc;
            const int gr = gcr, gz = gcz;
            const bool valid = coll;
            // uniform over the workgroup: no axis or wall row, no z wrap
            const bool plain = band_inner && R0 + SR * k >= 1 && R0 + SR * k + SR <= nr - 1;
            if (valid) {
                const int ux = lz + 2;
                C sig = C(0);  // sum of the stored values: rho - rho_ref when shifted
#pragma unroll
                for (int i = 0; i < kQ; ++i) sig += fc[i];
                const C rho = P::kShift ? sig + rho_ref : sig;
                const C jz = (fc[1] - fc[3]) + (fc[5] - fc[6]) + (fc[8] - fc[7]);
                const C jr = (fc[2] - fc[4]) + (fc[5] - fc[8]) + (fc[6] - fc[7]);
                const C uz = s_uz[wslot(l) * UW + ux], ur = s_ur[wslot(l) * UW + ux];
                const C rr = C(gr) + C(0.5);
                C hz = C(0), hr = C(0), mass = C(0);
                if (a.axisym) {
                    // H and the mass source (Eqs. H_terms, condition_h); the
                    // velocity derivatives read rows up to 2 away
                    const bool zd = no_wall_deriv && gr >= nr - 2;
                    const C druz = zd ? C(0) : d_r_win(s_uz, UW, NW - 1, l, ux);
                    const C dzur = zd ? C(0) : d_z_win(s_ur, UW, NW - 1, l, ux);
                    const C drur = zd ? C(0) : d_r_win(s_ur, UW, NW - 1, l, ux);
                    const C inv_r = dev_rcp(rr);
                    const C mu = rho * mu_fac;
                    hz = (mu * (druz + dzur) - rho * ur * uz) * inv_r;
                    hr = (C(2) * mu * (drur - ur * inv_r) - rho * ur * ur) * inv_r;
                    mass = -rho * ur * inv_r;
                }
                const C Fz = Fzc, Fr = Frc;
                const C inv_rho = dev_rcp(rho);
                const C qz = guo ? uz : (jz + tau * Fz) * inv_rho;
                const C qr = guo ? ur : (jr + tau * Fr) * inv_rho;
                const C qq = C(1.5) * (qz * qz + qr * qr);
                const C gpre = C(1) - C(0.5) * inv_tau;
                const C uF = uz * Fz + ur * Fr;
                constexpr bool kRem = sizeof(C) == 4;
                C feq_acc = C(0), h_acc = C(0);
#pragma unroll
                for (int ii = 0; ii < kQ; ++ii) {
                    const int i = kRem ? (ii + 1) % kQ : ii;
                    const C w = C(weight(i));
                    C feq, hi;
                    if (kRem && i == 0) {
                        feq = sig - feq_acc;
                        hi = mass - h_acc;
                    } else {
                        const C cu = C(cz(i)) * qz + C(cr(i)) * qr;
                        const C poly = C(3) * cu + C(4.5) * cu * cu - qq;
                        feq = P::kShift ? w * (sig + rho * poly) : w * rho * (C(1) + poly);
                        hi = w * (mass + C(3) * (C(cz(i)) * hz + C(cr(i)) * hr));
                        if (guo) {
                            const C cF = C(cz(i)) * Fz + C(cr(i)) * Fr;
                            const C cuu = C(cz(i)) * uz + C(cr(i)) * ur;
                            hi += gpre * w * (C(3) * (cF - uF) + C(9) * cuu * cF);
                        }
                        feq_acc += feq;
                        h_acc += hi;
                    }
                    fc[i] = fc[i] - (fc[i] - feq) * inv_tau + hi;
                }
                if (plain) {
                    const unsigned node_off = (unsigned)(gr * nz + gz) * (unsigned)sizeof(S);
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        const unsigned disp = (unsigned)((cr(i) * nz + cz(i)) * (int)sizeof(S));
                        buf_store<kStoreAux>(fout, node_off, (unsigned)i * plane_bytes + disp, S(fc[i]));
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        int tz = gz + cz(i), trr = gr + cr(i), d = i;
                        if (cr(i) < 0 && gr == 0) {
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
                                             S(fc[i]));
                    }
                }
            }
        }
        if (lr < 2) {
            Fzc = Fzn;
            Frc = Frn;
        }
    }
}

}  // namespace lbm
