// Hand-written adjoint (vector-Jacobian product) of one time step of the
// axisymmetric Shan–Chen scheme, FP64.
//
// Forward step (Sec. II): f* = C(f; G, tau), f_next = S(f*), with C the
// collision with all its force and source terms and S the push streaming
// with the boundary rules of Sec. II.E.  Given lam_next = dL/df_next the
// kernels below produce lam = (df_next/df)^T lam_next and accumulate
// dL/dG and dL/dtau.
//
// The reverse pass follows the forward data flow backwards:
//   1. forward intermediates at the current state are recomputed into
//      FP64 fields (rho, j, psi, d_r psi on the ghost-extended rows, d_rr,
//      the 1D d_r and d_zr, force, u, u^eq, velocity derivatives);
//   2. nu = S^T lam_next is gathered (S is a permutation);
//   3. the collision, equilibrium and source terms are reversed node by
//      node;
//   4. every stencil is transposed into a gather: the adjoint of a ghost
//      (mirrored) value is added back onto the real node it mirrors, with
//      the same parity sign the forward extension used;
//   5. psi-bar becomes rho-bar through psi'(rho) = exp(-rho/rho0), and
//      lam_i = f-bar_i + rho-bar + c_i . j-bar.
// Every kernel is one thread per node; no atomics, so results are
// deterministic.
#include <hip/hip_runtime.h>

#include <climits>

#include <cmath>
#include <map>
#include <mutex>
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

constexpr int NGA = 6;  // ghost rows kept on extended adjoint fields
// workgroup size of the per-node adjoint kernels: one wave per workgroup: a small lattice still spreads over every CU; the
// kernels declare it as their launch bound, which lets a thread keep all the
// loads of a gather in flight in registers
constexpr int kAdjBlock = 64;

struct AdjArgs {
    int nz, nr;
    long long n;    // nz * nr
    long long ne;   // nz * (nr + 2 NGA)
    double G, tau, rho0, gz;
    int wall, axisym;
    const double* f;         // [9][n] state f^t
    const double* lam_next;  // [9][n]
    double* lam;             // [9][n]
    double* fw;              // forward fields of the step (recomputed)
    double* w;               // adjoint fields, f-bar, partial sums
    int accumulate;          // 1: add the block partials of dL/dG, dL/dtau to running sums
};

// field slots (each n doubles): the forward ones (S_RHO .. S_QR) in a
// forward block, the adjoint ones (S_RHOB ..) in the adjoint block
enum Slot {
    S_RHO, S_JZ, S_JR, S_PSI, S_DRR, S_DZR, S_FZ, S_FR, S_SCZ, S_SCR, S_UZ, S_UR, S_QZ, S_QR,
    // adjoints
    S_RHOB, S_JZB, S_JRB, S_UZB_H, S_URB_H, S_FZB, S_FRB, S_DRUZB, S_DZURB, S_DRURB,
    S_PSIB_LOC, S_DZRB, S_DRRB, S_DRB_REAL, S_D1B, S_FSCZB, S_FSCRB, S_GB, S_TAUB,
    S_NSLOT
};
// extended slots (ne doubles each), after the plain ones of their block
// (E_PSI .. E_UR forward, E_DRB adjoint)
enum SlotE { E_PSI, E_DR, E_UZ, E_UR, E_DRB, E_NSLOT };
constexpr int kFwdSlots = S_RHOB, kFwdESlots = E_DRB;
// doubles in one forward block
__host__ __device__ inline size_t fwd_block(long long n, long long ne) {
    return (size_t)kFwdSlots * n + (size_t)kFwdESlots * ne;
}
// a slot's field inside its block
__device__ __forceinline__ double* fptr(const AdjArgs& a, int s) {
    return s < kFwdSlots ? a.fw + (size_t)s * a.n : a.w + (size_t)(s - kFwdSlots) * a.n;
}
__device__ __forceinline__ double* eptr(const AdjArgs& a, int s) {
    return s < kFwdESlots ? a.fw + (size_t)kFwdSlots * a.n + (size_t)s * a.ne
                          : a.w + (size_t)(S_NSLOT - kFwdSlots) * a.n + (size_t)(s - kFwdESlots) * a.ne;
}
// in the adjoint block, after its extended slot: the partial f-bar, a
// population-sized field
__host__ __device__ inline size_t fbar_off(long long n, long long ne) {
    return (size_t)(S_NSLOT - kFwdSlots) * n + (size_t)(E_NSLOT - kFwdESlots) * ne;
}
// after f-bar: per-block partial sums of dL/dG and dL/dtau ([block][2])
__host__ __device__ inline size_t part_off(long long n, long long ne) { return fbar_off(n, ne) + 9 * (size_t)n; }
// running per-block sums of a multi-step run, after the step partials
__host__ __device__ inline size_t run_off(long long n, long long ne) {
    return part_off(n, ne) + 2 * (size_t)((n + kAdjBlock - 1) / kAdjBlock);
}

// row clamped into [lo, hi] (the masked gathers below load a clamped row and
// multiply its term by 0 when the row is outside: no branch around the load)
__device__ __forceinline__ int clampi(int y, int lo, int hi) { return y < lo ? lo : (y > hi ? hi : y); }

// periodic column: the stencils here reach at most 2 columns and the
// adjoint requires nz >= 4, so one add or subtract wraps
__device__ __forceinline__ int wrapz(int z, int nz) {
    z = z < 0 ? z + nz : z;
    return z >= nz ? z - nz : z;
}
__device__ __forceinline__ int mirror_src(int y, int nr, double& sgn, double axis_sign) {
    sgn = 1.0;
    if (y < 0) {
        sgn = axis_sign;
        return -1 - y;
    }
    if (y >= nr) return 2 * nr - 1 - y;
    return y;
}
// extended-field index of row y (-NGA <= y < nr + NGA), column z
__device__ __forceinline__ long long eidx(int y, int z, int nz) { return (long long)(y + NGA) * nz + z; }

#define NODE_LOOP(a)                                                 \
    const long long x = gid;                                         \
    if (x >= (a).n) return;                                          \
    const int r = (int)x / (a).nz, z = (int)x - r * (a).nz;

// isotropic first derivative at (z, y) of an extended field (Sec. II.D)
__device__ double d_iso_e(const double* E, int z, int y, int nz, bool along_r) {
    double s = 0.0;
#pragma unroll
    for (int i = 1; i < lbm::kQ; ++i) {
        const int c = along_r ? lbm::cr(i) : lbm::cz(i);
        if (c == 0) continue;
        const double t = 8.0 * E[eidx(y + lbm::cr(i), wrapz(z + lbm::cz(i), nz), nz)] -
                         E[eidx(y + 2 * lbm::cr(i), wrapz(z + 2 * lbm::cz(i), nz), nz)];
        s += c * t;
    }
    return s / 36.0;
}

// ------------------------------------------------------------ forward ----

// rho, j, psi on the real rows and psi on the extended rows -6 .. nr+5
// (a ghost row takes the value of its mirror row: psi is even at the axis
// and at the wall)
__device__ __forceinline__ void fwd_moments_at(const AdjArgs& a, const long long gid) {
    const long long e = gid;
    if (e >= a.ne) return;
    const int y = (int)e / a.nz - NGA, z = (int)e - (y + NGA) * a.nz;
    double sgn;
    const int ys = mirror_src(y, a.nr, sgn, 1.0);
    double* w = a.w;
    const long long n = a.n;
    const long long x = (long long)ys * a.nz + z;
    double rho = 0, jz = 0, jr = 0;
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) {
        const double fi = a.f[i * n + x];
        rho += fi;
        jz += lbm::cz(i) * fi;
        jr += lbm::cr(i) * fi;
    }
    const double psi = a.rho0 * (1.0 - exp(-rho / a.rho0));
    if (y == ys) {
        fptr(a, S_RHO)[x] = rho;
        fptr(a, S_JZ)[x] = jz;
        fptr(a, S_JR)[x] = jr;
        fptr(a, S_PSI)[x] = psi;
    }
    eptr(a, E_PSI)[e] = psi;
}

// isotropic d_r psi on extended rows -4 .. nr+3 (zero elsewhere)
__device__ __forceinline__ void fwd_dr_at(const AdjArgs& a, const long long gid) {
    const long long e = gid;
    if (e >= a.ne) return;
    const int y = (int)e / a.nz - NGA, z = (int)e - (y + NGA) * a.nz;
    const double* psiE = eptr(a, E_PSI);
    double v = 0.0;
    if (y >= -4 && y < a.nr + 4) v = d_iso_e(psiE, z, y, a.nz, true);
    eptr(a, E_DR)[e] = v;
}

// forces, hydrodynamic and equilibrium velocities on the real rows, and the
// velocity on the extended rows (a ghost row recomputes its mirror row's
// value: u_z even, u_r odd at the axis and even at the wall)
__device__ __forceinline__ void fwd_force_at(const AdjArgs& a, const long long gid) {
    const long long e = gid;
    if (e >= a.ne) return;
    const int y = (int)e / a.nz - NGA, z = (int)e - (y + NGA) * a.nz;
    double sgn;
    const int r = mirror_src(y, a.nr, sgn, -1.0);
    double* w = a.w;
    const long long n = a.n;
    const int nz = a.nz;
    const long long x = (long long)r * nz + z;
    const double* psiE = eptr(a, E_PSI);
    const double* drE = eptr(a, E_DR);
    // 1D fourth-order d_z of the 1D fourth-order d_r (Sec. II.D)
    auto d1 = [&](int zz) {
        zz = wrapz(zz, nz);
        return (-psiE[eidx(r + 2, zz, nz)] + 8.0 * psiE[eidx(r + 1, zz, nz)] - 8.0 * psiE[eidx(r - 1, zz, nz)] +
                psiE[eidx(r - 2, zz, nz)]) / 12.0;
    };
    const double dzr = (-d1(z + 2) + 8.0 * d1(z + 1) - 8.0 * d1(z - 1) + d1(z - 2)) / 12.0;
    const double drr = d_iso_e(drE, z, r, nz, true);
    double sz = 0, sr = 0;
#pragma unroll
    for (int i = 1; i < lbm::kQ; ++i) {
        const double ps = psiE[eidx(r + lbm::cr(i), wrapz(z + lbm::cz(i), nz), nz)];
        sz += lbm::weight(i) * ps * lbm::cz(i);
        sr += lbm::weight(i) * ps * lbm::cr(i);
    }
    const double psi = fptr(a, S_PSI)[x], rho = fptr(a, S_RHO)[x];
    double Fz = -a.G * psi * sz, Fr = -a.G * psi * sr;
    if (a.axisym) {
        const double rr = r + 0.5;
        const double dr1 = drE[eidx(r, z, nz)];
        Fz += -(a.G / 18.0) * psi * dzr / rr;
        Fr += -(a.G / 18.0) * psi * (drr / rr - dr1 / (rr * rr));
    }
    Fz += rho * a.gz;
    const double jz = fptr(a, S_JZ)[x], jr = fptr(a, S_JR)[x];
    const double uz = (jz + 0.5 * Fz) / rho, ur = (jr + 0.5 * Fr) / rho;
    if (y == r) {
        fptr(a, S_DZR)[x] = dzr;
        fptr(a, S_DRR)[x] = drr;
        fptr(a, S_SCZ)[x] = sz;
        fptr(a, S_SCR)[x] = sr;
        fptr(a, S_FZ)[x] = Fz;
        fptr(a, S_FR)[x] = Fr;
        fptr(a, S_UZ)[x] = uz;
        fptr(a, S_UR)[x] = ur;
        fptr(a, S_QZ)[x] = (jz + a.tau * Fz) / rho;
        fptr(a, S_QR)[x] = (jr + a.tau * Fr) / rho;
    }
    eptr(a, E_UZ)[e] = uz;
    eptr(a, E_UR)[e] = sgn * ur;
}

// ------------------------------------------------------------ reverse ----


// steps 2-3: streaming transpose, BGK / equilibrium / source reversed.
// kIn: a row with no boundary link (1 <= r <= nr - 2), whose push targets
// need no boundary rule, so the loop's loads carry no branches.
// kAxi: the axisymmetric terms (a.axisym), a template flag so that no branch
// separates the velocity-stencil loads from the others
template <bool kIn, bool kAxi>
__device__ __forceinline__ void rev_collision_node(const AdjArgs& a, const long long x, const int r, const int z) {
    double* w = a.w;
    const long long n = a.n;
    const double tau = a.tau, inv_tau = 1.0 / tau;
    const double rho = fptr(a, S_RHO)[x];
    const double qz = fptr(a, S_QZ)[x], qr = fptr(a, S_QR)[x];
    const double uz = fptr(a, S_UZ)[x], ur = fptr(a, S_UR)[x];
    const double rr = r + 0.5;
    double* fbar = w + fbar_off(n, a.ne);

    double rhob = 0, qzb = 0, qrb = 0, taub = 0, massb = 0, hzb = 0, hrb = 0;
    const double qq = 1.5 * (qz * qz + qr * qr);
    // every load first: the f-bar stores below could alias them for all the
    // compiler knows, and would otherwise make each load wait in turn
    double druz = 0, dzur = 0, drur = 0;
    if (kAxi) {
        const double* uzE = eptr(a, E_UZ);
        const double* urE = eptr(a, E_UR);
        druz = d_iso_e(uzE, z, r, a.nz, true);
        dzur = d_iso_e(urE, z, r, a.nz, false);
        drur = d_iso_e(urE, z, r, a.nz, true);
    }
    const double Fz = fptr(a, S_FZ)[x], Fr = fptr(a, S_FR)[x];
    double nus[lbm::kQ], fis[lbm::kQ];
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) {
        int tz, tr, d;
        if (kIn) {
            tz = wrapz(z + lbm::cz(i), a.nz);
            tr = r + lbm::cr(i);
            d = i;
        } else {
            // the push target under the boundary rules (Sec. II.E: the
            // specular axis, the no-slip or free-slip wall), as selects so
            // that no branch separates the loads
            const int ty = r + lbm::cr(i);
            const bool below = ty < 0, above = ty >= a.nr, back = above && a.wall == 0;
            tz = wrapz(back ? z : z + lbm::cz(i), a.nz);
            tr = below ? 0 : (above ? (a.wall == 0 ? r : a.nr - 1) : ty);
            d = below ? lbm::mirror_r(i) : (above ? (a.wall == 0 ? lbm::opposite(i) : lbm::mirror_r(i)) : i);
        }
        nus[i] = a.lam_next[d * n + (long long)tr * a.nz + tz];
        fis[i] = a.f[i * n + x];
    }
#pragma unroll
    for (int i = 0; i < lbm::kQ; ++i) {
        const double nu = nus[i];
        const double wi = lbm::weight(i);
        const double cu = lbm::cz(i) * qz + lbm::cr(i) * qr;
        const double poly = 3.0 * cu + 4.5 * cu * cu - qq;
        const double feq = wi * rho * (1.0 + poly);
        const double fi = fis[i];
        fbar[i * n + x] = nu * (1.0 - inv_tau);
        taub += nu * (fi - feq) * inv_tau * inv_tau;
        const double feqb = nu * inv_tau;
        rhob += feqb * wi * (1.0 + poly);
        const double dpoly = wi * rho * feqb * (3.0 + 9.0 * cu);  // d feq / d cu
        qzb += dpoly * lbm::cz(i) - feqb * wi * rho * 3.0 * qz;
        qrb += dpoly * lbm::cr(i) - feqb * wi * rho * 3.0 * qr;
        massb += wi * nu;
        hzb += 3.0 * wi * lbm::cz(i) * nu;
        hrb += 3.0 * wi * lbm::cr(i) * nu;
    }
    double uzb = 0, urb = 0, druzb = 0, dzurb = 0, drurb = 0;
    if (kAxi) {
        const double mu = rho * (tau - 0.5) / 3.0;
        // mass = -rho u_r / r
        rhob += -massb * ur / rr;
        urb += -massb * rho / rr;
        // H_z = (mu (d_r u_z + d_z u_r) - rho u_r u_z) / r
        double mub = hzb * (druz + dzur) / rr;
        druzb += hzb * mu / rr;
        dzurb += hzb * mu / rr;
        rhob += -hzb * ur * uz / rr;
        urb += -hzb * rho * uz / rr;
        uzb += -hzb * rho * ur / rr;
        // H_r = (2 mu (d_r u_r - u_r / r) - rho u_r^2) / r
        mub += hrb * 2.0 * (drur - ur / rr) / rr;
        drurb += hrb * 2.0 * mu / rr;
        urb += hrb * (-2.0 * mu / (rr * rr) - 2.0 * rho * ur / rr);
        rhob += -hrb * ur * ur / rr;
        // mu = rho (tau - 1/2) / 3
        rhob += mub * (tau - 0.5) / 3.0;
        taub += mub * rho / 3.0;
    }
    // u^eq = (j + tau F) / rho
    const double jzb = qzb / rho, jrb = qrb / rho;
    const double Fzb = tau * qzb / rho, Frb = tau * qrb / rho;
    taub += (qzb * Fz + qrb * Fr) / rho;
    rhob += -(qzb * qz + qrb * qr) / rho;
    fptr(a, S_RHOB)[x] = rhob;
    fptr(a, S_JZB)[x] = jzb;
    fptr(a, S_JRB)[x] = jrb;
    fptr(a, S_FZB)[x] = Fzb;
    fptr(a, S_FRB)[x] = Frb;
    fptr(a, S_UZB_H)[x] = uzb;
    fptr(a, S_URB_H)[x] = urb;
    fptr(a, S_DRUZB)[x] = druzb;
    fptr(a, S_DZURB)[x] = dzurb;
    fptr(a, S_DRURB)[x] = drurb;
    fptr(a, S_TAUB)[x] = taub;
}
__device__ __forceinline__ void rev_collision_at(const AdjArgs& a, const long long gid) {
    NODE_LOOP(a)
    const bool in = r >= 1 && r <= a.nr - 2;
    if (a.axisym) {
        if (in)
            rev_collision_node<true, true>(a, x, r, z);
        else
            rev_collision_node<false, true>(a, x, r, z);
    } else {
        if (in)
            rev_collision_node<true, false>(a, x, r, z);
        else
            rev_collision_node<false, false>(a, x, r, z);
    }
}

// transposed isotropic stencil: sum over taps o of coef(o) * src(e - o),
// src living on real rows of a plain field.  kAll: every tap row is a real
// row and the taps are summed as they are; otherwise a tap outside the
// lattice loads a clamped row and is multiplied by 0.  Either way no branch
// surrounds a load, so a thread issues them all before waiting on any (a
// check around each load makes each wait for the previous one).
template <bool kAll>
__device__ double iso_transpose_real_t(const double* src, int z, int e, int nz, int nr, bool along_r) {
    double s = 0.0;
#pragma unroll
    for (int i = 1; i < lbm::kQ; ++i) {
        const int c = along_r ? lbm::cr(i) : lbm::cz(i);
        if (c == 0) continue;
        const int y1 = e - lbm::cr(i), y2 = e - 2 * lbm::cr(i);
        if (kAll) {
            s += 8.0 * c * src[(long long)y1 * nz + wrapz(z - lbm::cz(i), nz)];
            s -= c * src[(long long)y2 * nz + wrapz(z - 2 * lbm::cz(i), nz)];
        } else {
            // masked: a row outside the lattice contributes 0 x (a real value)
            const double m1 = (y1 >= 0 && y1 < nr) ? 1.0 : 0.0, m2 = (y2 >= 0 && y2 < nr) ? 1.0 : 0.0;
            s += 8.0 * c * m1 * src[(long long)clampi(y1, 0, nr - 1) * nz + wrapz(z - lbm::cz(i), nz)];
            s -= c * m2 * src[(long long)clampi(y2, 0, nr - 1) * nz + wrapz(z - 2 * lbm::cz(i), nz)];
        }
    }
    return s / 36.0;
}
__device__ double iso_transpose_real(const double* src, int z, int e, int nz, int nr, bool along_r) {
    return (e >= 2 && e <= nr - 3) ? iso_transpose_real_t<true>(src, z, e, nz, nr, along_r)
                                   : iso_transpose_real_t<false>(src, z, e, nz, nr, along_r);
}

// step 4 for the velocities, then u = (j + F/2)/rho and the force reversed
__device__ __forceinline__ void rev_velocity_force_at(const AdjArgs& a, const long long gid) {
    NODE_LOOP(a)
    double* w = a.w;
    const long long n = a.n;
    const int nz = a.nz, nr = a.nr;
    double uzb = fptr(a, S_UZB_H)[x], urb = fptr(a, S_URB_H)[x];
    // the node's own fields, loaded together with the gathers below
    const double rho = fptr(a, S_RHO)[x];
    const double uz = fptr(a, S_UZ)[x], ur = fptr(a, S_UR)[x];
    const double jzb0 = fptr(a, S_JZB)[x], jrb0 = fptr(a, S_JRB)[x];
    const double Fzb0 = fptr(a, S_FZB)[x], Frb0 = fptr(a, S_FRB)[x];
    const double rhob0 = fptr(a, S_RHOB)[x];
    const double psi = fptr(a, S_PSI)[x];
    const double sz = fptr(a, S_SCZ)[x], sr = fptr(a, S_SCR)[x];
    const double dzr = fptr(a, S_DZR)[x], drr = fptr(a, S_DRR)[x];
    const double dr1 = eptr(a, E_DR)[eidx(r, z, nz)];
    if (a.axisym) {
        // images of row r in the extended velocity fields (reach 2)
        const double* druzb = fptr(a, S_DRUZB);
        const double* dzurb = fptr(a, S_DZURB);
        const double* drurb = fptr(a, S_DRURB);
        // one interior test for the three gathers of an image row, so that
        // their loads go out together
        auto gather = [&](int e, double sgn_r) {
            if (e >= 2 && e <= nr - 3) {
                uzb += iso_transpose_real_t<true>(druzb, z, e, nz, nr, true);
                urb += sgn_r * (iso_transpose_real_t<true>(dzurb, z, e, nz, nr, false) +
                                iso_transpose_real_t<true>(drurb, z, e, nz, nr, true));
            } else {
                uzb += iso_transpose_real_t<false>(druzb, z, e, nz, nr, true);
                urb += sgn_r * (iso_transpose_real_t<false>(dzurb, z, e, nz, nr, false) +
                                iso_transpose_real_t<false>(drurb, z, e, nz, nr, true));
            }
        };
        gather(r, 1.0);
        if (r <= 1) gather(-1 - r, -1.0);          // axis image: u_r odd
        if (r >= nr - 2) gather(2 * nr - 1 - r, 1.0);  // wall image
    }
    double jzb = jzb0 + uzb / rho;
    double jrb = jrb0 + urb / rho;
    double Fzb = Fzb0 + 0.5 * uzb / rho;
    double Frb = Frb0 + 0.5 * urb / rho;
    double rhob = rhob0 - (uzb * uz + urb * ur) / rho;
    // F = F^SC + F^sym + rho g z^
    rhob += Fzb * a.gz;
    double Gb = -psi * (Fzb * sz + Frb * sr);
    double psib = -a.G * (Fzb * sz + Frb * sr);
    double dzrb = 0, drrb = 0, dr1b = 0;
    if (a.axisym) {
        const double rr = r + 0.5;
        const double g18 = a.G / 18.0;
        // F^sym_z = -(G/18) psi d_zr / r
        Gb += Fzb * (-psi * dzr / (18.0 * rr));
        psib += Fzb * (-g18 * dzr / rr);
        dzrb = Fzb * (-g18 * psi / rr);
        // F^sym_r = -(G/18) psi (d_rr / r - d_r / r^2)
        const double br = drr / rr - dr1 / (rr * rr);
        Gb += Frb * (-psi * br / 18.0);
        psib += Frb * (-g18 * br);
        drrb = Frb * (-g18 * psi / rr);
        dr1b = Frb * (g18 * psi / (rr * rr));
    }
    fptr(a, S_JZB)[x] = jzb;
    fptr(a, S_JRB)[x] = jrb;
    fptr(a, S_RHOB)[x] = rhob;
    fptr(a, S_FSCZB)[x] = Fzb;  // adjoint of F^SC equals that of F
    fptr(a, S_FSCRB)[x] = Frb;
    fptr(a, S_PSIB_LOC)[x] = psib;
    fptr(a, S_DZRB)[x] = dzrb;
    fptr(a, S_DRRB)[x] = drrb;
    fptr(a, S_DRB_REAL)[x] = dr1b;
    fptr(a, S_GB)[x] = Gb;
}

// Two independent transposed stencils in one pass (both read only what
// rev_velocity_force wrote):
// - adjoint of d_r psi on extended rows -2 .. nr+1 (the rows d_rr reads):
//   transposed d_rr plus the direct use of d_r on real rows;
// - on real rows, d_zr = 1D d_z of the 1D d_r: transpose of the outer z
//   difference.
__device__ __forceinline__ void rev_dr_at(const AdjArgs& a, const long long gid) {
    const long long e = gid;
    if (e >= a.ne) return;
    const int y = (int)e / a.nz - NGA, z = (int)e - (y + NGA) * a.nz;
    const int nz = a.nz;
    double v = 0.0;
    if (y >= -2 && y < a.nr + 2) {
        v = iso_transpose_real(fptr(a, S_DRRB), z, y, nz, a.nr, true);
        if (y >= 0 && y < a.nr) v += fptr(a, S_DRB_REAL)[(long long)y * nz + z];
    }
    eptr(a, E_DRB)[e] = v;
    if (y >= 0 && y < a.nr) {
        const double* b = fptr(a, S_DZRB) + (long long)y * nz;
        // forward: out(z) = (-in(z+2) + 8 in(z+1) - 8 in(z-1) + in(z-2)) / 12
        fptr(a, S_D1B)[(long long)y * nz + z] =
            (-b[wrapz(z - 2, nz)] + 8.0 * b[wrapz(z - 1, nz)] - 8.0 * b[wrapz(z + 1, nz)] + b[wrapz(z + 2, nz)]) /
            12.0;
    }
}

__device__ __forceinline__ long long global_id() { return (long long)blockIdx.x * blockDim.x + threadIdx.x; }

__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void fwd_moments(AdjArgs a) { fwd_moments_at(a, global_id()); }
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void fwd_dr(AdjArgs a) { fwd_dr_at(a, global_id()); }
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void fwd_force(AdjArgs a) { fwd_force_at(a, global_id()); }
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void rev_collision(AdjArgs a) { rev_collision_at(a, global_id()); }
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void rev_velocity_force(AdjArgs a) { rev_velocity_force_at(a, global_id()); }
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void rev_dr(AdjArgs a) { rev_dr_at(a, global_id()); }

// In a run, the reverse kernels of step t share their launches with the
// recomputation of step t - 1, whose fields go to the other forward block:
// the two parts of a launch touch no common field.  (Giving the two parts
// separate workgroups of one launch, or issuing the recomputation's loads
// ahead of the reverse part, was no faster.)
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void rev_collision_fwd_moments(AdjArgs ar, AdjArgs af, int fwd) {
    const long long g = global_id();
    rev_collision_at(ar, g);
    if (fwd) fwd_moments_at(af, g);
}
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void rev_velocity_force_fwd_dr(AdjArgs ar, AdjArgs af, int fwd) {
    const long long g = global_id();
    rev_velocity_force_at(ar, g);
    if (fwd) fwd_dr_at(af, g);
}
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void rev_dr_fwd_force(AdjArgs ar, AdjArgs af, int fwd) {
    const long long g = global_id();
    rev_dr_at(ar, g);
    if (fwd) fwd_force_at(af, g);
}

// adjoint of extended psi at extended row e, column z (before folding);
// kAll: 2 <= e <= nr - 3, every tap of the three gathers lies inside
template <bool kAll>
__device__ double psi_ext_adjoint_t(const AdjArgs& a, int z, int e) {
    const double* w = a.w;
    const long long n = a.n;
    const int nz = a.nz, nr = a.nr;
    double s = 0.0;
    // d_r psi = iso_r(psi_ext) on rows -4..nr+3; only rows -2..nr+1 carry adjoint
    const double* drb = eptr(a, E_DRB);
#pragma unroll
    for (int i = 1; i < lbm::kQ; ++i) {
        const int c = lbm::cr(i);
        if (c == 0) continue;
        // every tap row lies inside the extended field (|e| reaches at most 4
        // beyond the lattice, the field 6), whose rows outside -2 .. nr+1
        // hold zeros: no test is needed
        const int y1 = e - lbm::cr(i), y2 = e - 2 * lbm::cr(i);
        s += (8.0 * c / 36.0) * drb[eidx(y1, wrapz(z - lbm::cz(i), nz), nz)];
        s -= (c / 36.0) * drb[eidx(y2, wrapz(z - 2 * lbm::cz(i), nz), nz)];
    }
    // 1D d_r psi on real rows: (-p(y+2) + 8 p(y+1) - 8 p(y-1) + p(y-2)) / 12
    const double* d1b = fptr(a, S_D1B);
    const int ys[4] = {e - 2, e - 1, e + 1, e + 2};
    const double cf[4] = {-1.0, 8.0, -8.0, 1.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (kAll) {
            s += (cf[k] / 12.0) * d1b[(long long)ys[k] * nz + z];
        } else {
            const double m = (ys[k] >= 0 && ys[k] < nr) ? 1.0 : 0.0;
            s += (cf[k] / 12.0) * m * d1b[(long long)clampi(ys[k], 0, nr - 1) * nz + z];
        }
    }
    // Shan–Chen force: F^SC(x) = -G psi(x) sum_i W_i psi(x + c_i) c_i
    const double* fzb = fptr(a, S_FSCZB);
    const double* frb = fptr(a, S_FSCRB);
    const double* psi = fptr(a, S_PSI);
#pragma unroll
    for (int i = 1; i < lbm::kQ; ++i) {
        const int ysrc = e - lbm::cr(i);
        const double m = (kAll || (ysrc >= 0 && ysrc < nr)) ? 1.0 : 0.0;
        const long long xs = (long long)(kAll ? ysrc : clampi(ysrc, 0, nr - 1)) * nz + wrapz(z - lbm::cz(i), nz);
        s += -a.G * psi[xs] * lbm::weight(i) * m * (fzb[xs] * lbm::cz(i) + frb[xs] * lbm::cr(i));
    }
    return s;
}
__device__ double psi_ext_adjoint(const AdjArgs& a, int z, int e) {
    return (e >= 2 && e <= a.nr - 3) ? psi_ext_adjoint_t<true>(a, z, e) : psi_ext_adjoint_t<false>(a, z, e);
}

// step 4 for psi (fold every image of the row), step 5, write lam
// Last reverse kernel: lam = f-bar + rho-bar + c . j-bar, and the block's
// partial sums of the node contributions to dL/dG and dL/dtau (a fixed
// tree order, so the result does not depend on scheduling).
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(1, 2))) void rev_psi_final(AdjArgs a) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double* w = a.w;
    const long long n = a.n;
    double g = 0.0, q = 0.0;
    if (x < n) {
        const int nr = a.nr;
        const int r = (int)x / a.nz, z = (int)x - r * a.nz;
        // the node's own fields first, so that no load waits behind the
        // stores of lam (which could alias them for all the compiler knows)
        const double psib_loc = fptr(a, S_PSIB_LOC)[x];
        const double rho = fptr(a, S_RHO)[x], rhob_loc = fptr(a, S_RHOB)[x];
        const double jzb = fptr(a, S_JZB)[x], jrb = fptr(a, S_JRB)[x];
        const double* fbar = w + fbar_off(n, a.ne);
        double fb[lbm::kQ];
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) fb[i] = fbar[i * n + x];
        g = fptr(a, S_GB)[x];
        q = fptr(a, S_TAUB)[x];
        double psib = psib_loc + psi_ext_adjoint(a, z, r);
        if (r <= 3) psib += psi_ext_adjoint(a, z, -1 - r);            // axis images (rows -4..-1)
        if (r >= nr - 4) psib += psi_ext_adjoint(a, z, 2 * nr - 1 - r);  // wall images (rows nr..nr+3)
        const double rhob = rhob_loc + psib * exp(-rho / a.rho0);
#pragma unroll
        for (int i = 0; i < lbm::kQ; ++i) a.lam[i * n + x] = fb[i] + rhob + lbm::cz(i) * jzb + lbm::cr(i) * jrb;
    }
    // the workgroup is one wave: a tree of lane shuffles, lane 0 adding
    // lane k's value for k = 32, 16, ..., 1 (a fixed order)
    static_assert(kAdjBlock == 64, "one wave per workgroup");
    const int t = threadIdx.x;
#pragma unroll
    for (int k = kAdjBlock / 2; k > 0; k >>= 1) {
        g += __shfl_down(g, k, 64);
        q += __shfl_down(q, k, 64);
    }
    if (t == 0) {
        // one step: this step's partials; a run: the block's running sums
        // over its steps, in step order
        const size_t o = (a.accumulate ? run_off(n, a.ne) : part_off(n, a.ne)) + 2 * (size_t)blockIdx.x;
        if (a.accumulate) {
            w[o] += g;
            w[o + 1] += q;
        } else {
            w[o] = g;
            w[o + 1] = q;
        }
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

// workspace: two forward blocks (a run recomputes step t - 1 into one while
// step t is reversed from the other), then the adjoint block
AdjArgs adjoint_args(const lbm_axi_params* p, void* d_ws, int accumulate, int parity = 0) {
    AdjArgs a{};
    a.nz = p->nz;
    a.nr = p->nr;
    a.n = (long long)p->nz * p->nr;
    a.ne = (long long)p->nz * (p->nr + 2 * NGA);
    a.G = p->G;
    a.tau = p->tau;
    a.rho0 = p->psi_rho0;
    a.gz = p->gz;
    a.wall = p->wall;
    a.axisym = p->axisym;
    double* base = static_cast<double*>(d_ws);
    a.fw = base + (size_t)parity * fwd_block(a.n, a.ne);
    a.w = base + 2 * fwd_block(a.n, a.ne);
    a.accumulate = accumulate;
    return a;
}

int nparts_of(const AdjArgs& a) { return (int)((a.n + kAdjBlock - 1) / kAdjBlock); }

// the kernels of one reverse step, in order
void launch_reverse_step(AdjArgs a, const double* f, const double* lam_next, double* lam, hipStream_t s) {
    a.f = f;
    a.lam_next = lam_next;
    a.lam = lam;
    const dim3 b(kAdjBlock);
    const int bn = nparts_of(a), be = (int)((a.ne + kAdjBlock - 1) / kAdjBlock);
    hipLaunchKernelGGL(fwd_moments, dim3(be), b, 0, s, a);
    hipLaunchKernelGGL(fwd_dr, dim3(be), b, 0, s, a);
    hipLaunchKernelGGL(fwd_force, dim3(be), b, 0, s, a);
    hipLaunchKernelGGL(rev_collision, dim3(bn), b, 0, s, a);
    hipLaunchKernelGGL(rev_velocity_force, dim3(bn), b, 0, s, a);
    hipLaunchKernelGGL(rev_dr, dim3(be), b, 0, s, a);
    hipLaunchKernelGGL(rev_psi_final, dim3(bn), b, 0, s, a);
}

int check_adjoint(const lbm_axi_params* p, size_t ws_bytes) {
    if (!p) return LBM_AXI_EINVAL;
    if (p->nz < 4 || p->nr < 6 || !(p->tau > 0.5) || !(p->psi_rho0 > 0.0)) return LBM_AXI_EINVAL;
    // node indices are split with 32-bit arithmetic
    if ((long long)p->nz * (p->nr + 2 * NGA) > INT_MAX) return LBM_AXI_EINVAL;
    if (p->wall != 0 && p->wall != 1) return LBM_AXI_EINVAL;
    if (p->precision != LBM_AXI_FP64 || p->flags != 0) return LBM_AXI_EUNSUP;
    if (ws_bytes < lbm_axi_adjoint_workspace_bytes(p->nz, p->nr)) return LBM_AXI_ENOMEM;
    return LBM_AXI_OK;
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
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // the kernels overwrite every field and partial sum of one step before
    // reading it, so nothing needs clearing
    AdjArgs a = adjoint_args(p, ws, 0);
    launch_reverse_step(a, d_f, d_lam_next, d_lam, s);
    if (d_grad_acc)
        hipLaunchKernelGGL(rev_reduce, dim3(1), dim3(256), 0, s, a.w + part_off(a.n, a.ne), nparts_of(a), d_grad_acc);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_AXI_OK : lbm_host::hip_fail(e, "adjoint kernel launch");
}

size_t lbm_axi_adjoint_workspace_bytes(int32_t nz, int32_t nr) {
    if (nz < 4 || nr < 6 || (long long)nz * (nr + 2 * NGA) > INT_MAX) return 0;
    const long long n = (long long)nz * nr, ne = (long long)nz * (nr + 2 * NGA);
    const size_t nparts = (size_t)((n + kAdjBlock - 1) / kAdjBlock);
    return (2 * fwd_block(n, ne) + fbar_off(n, ne) + 9 * (size_t)n + 4 * nparts) * sizeof(double);
}

int lbm_axi_adjoint_step(const lbm_axi_params* p, const double* d_f, const double* d_lam_next, double* d_lam,
                         double* d_grad_acc, void* d_ws, size_t ws_bytes, void* hip_stream) {
    if (!p || !d_f || !d_lam_next || !d_lam || !d_ws) return LBM_AXI_EINVAL;
    const int rc = check_adjoint(p, ws_bytes);
    if (rc != LBM_AXI_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    AdjArgs a = adjoint_args(p, d_ws, 0);
    launch_reverse_step(a, d_f, d_lam_next, d_lam, s);
    if (d_grad_acc)
        hipLaunchKernelGGL(rev_reduce, dim3(1), dim3(256), 0, s, a.w + part_off(a.n, a.ne), nparts_of(a), d_grad_acc);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_adjoint_run(const lbm_axi_params* p, const double* d_states, int32_t k, double* d_lam, double* d_tmp,
                        double* d_grad_acc, void* d_ws, size_t ws_bytes, void* hip_stream) {
    if (!p || !d_states || !d_lam || !d_tmp || d_tmp == d_lam || !d_ws || k < 0) return LBM_AXI_EINVAL;
    const int rc = check_adjoint(p, ws_bytes);
    if (rc != LBM_AXI_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t n9 = 9 * (size_t)p->nz * (size_t)p->nr;
    AdjArgs a = adjoint_args(p, d_ws, 1);
    double* run = a.w + run_off(a.n, a.ne);
    const int nparts = nparts_of(a);
    // the block sums of dL/dG, dL/dtau run over the k steps and are reduced
    // once at the end (a kernel, not a memset, clears them)
    hipLaunchKernelGGL(zero_kernel, dim3(nblk(2 * (long long)nparts)), dim3(256), 0, s, run, 2 * (long long)nparts);
    const dim3 b(kAdjBlock);
    const int bn = nparts, be = (int)((a.ne + kAdjBlock - 1) / kAdjBlock);
    double* cur = d_lam;  // holds lam^{t0+j+1} before step j
    double* nxt = d_tmp;
    if (k > 0) {
        // fields of the last state, into forward block 0
        AdjArgs f0 = adjoint_args(p, d_ws, 1, 0);
        f0.f = d_states + (size_t)(k - 1) * n9;
        hipLaunchKernelGGL(fwd_moments, dim3(be), b, 0, s, f0);
        hipLaunchKernelGGL(fwd_dr, dim3(be), b, 0, s, f0);
        hipLaunchKernelGGL(fwd_force, dim3(be), b, 0, s, f0);
    }
    int par = 0;
    for (int32_t j = k - 1; j >= 0; --j) {
        AdjArgs ar = adjoint_args(p, d_ws, 1, par);  // step j, fields in block par
        ar.f = d_states + (size_t)j * n9;
        ar.lam_next = cur;
        ar.lam = nxt;
        AdjArgs af = adjoint_args(p, d_ws, 1, 1 - par);  // step j - 1, into the other block
        const int fwd = j > 0 ? 1 : 0;
        af.f = fwd ? d_states + (size_t)(j - 1) * n9 : nullptr;
        hipLaunchKernelGGL(rev_collision_fwd_moments, dim3(be), b, 0, s, ar, af, fwd);
        hipLaunchKernelGGL(rev_velocity_force_fwd_dr, dim3(be), b, 0, s, ar, af, fwd);
        hipLaunchKernelGGL(rev_dr_fwd_force, dim3(be), b, 0, s, ar, af, fwd);
        hipLaunchKernelGGL(rev_psi_final, dim3(bn), b, 0, s, ar);
        double* t = cur;
        cur = nxt;
        nxt = t;
        par = 1 - par;
    }
    if (d_grad_acc && k > 0) hipLaunchKernelGGL(rev_reduce, dim3(1), dim3(256), 0, s, run, nparts, d_grad_acc);
    if (hipGetLastError() != hipSuccess) return LBM_AXI_EHIP;
    if (cur != d_lam && hipMemcpyAsync(d_lam, cur, n9 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return LBM_AXI_EHIP;
    return LBM_AXI_OK;
}

int lbm_axi_init_vjp(const double* d_lam0, const double* d_uz0, const double* d_ur0, int32_t nz, int32_t nr,
                     double* d_rho0_bar, void* hip_stream) {
    if (!d_lam0 || !d_rho0_bar || nz < 1 || nr < 1) return LBM_AXI_EINVAL;
    const long long n = (long long)nz * nr;
    hipLaunchKernelGGL(init_vjp_kernel, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_lam0,
                       d_uz0, d_ur0, n, d_rho0_bar);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_density(const double* d_f, int32_t nz, int32_t nr, double* d_rho, void* hip_stream) {
    if (!d_f || !d_rho || nz < 1 || nr < 1) return LBM_AXI_EINVAL;
    const long long n = (long long)nz * nr;
    hipLaunchKernelGGL(density_kernel, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_f, n, d_rho);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_ray_forward(const double* d_rho, int32_t n_rows, const int32_t* d_row_ptr, const int32_t* d_col,
                        const double* d_val, double rho_l, double rho_g, double* d_out, void* hip_stream) {
    if (!d_rho || !d_row_ptr || !d_col || !d_val || !d_out || n_rows < 0 || rho_l == rho_g) return LBM_AXI_EINVAL;
    if (n_rows == 0) return LBM_AXI_OK;
    hipLaunchKernelGGL(ray_forward_kernel, dim3(n_rows), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_rho,
                       d_row_ptr, d_col, d_val, rho_l, rho_g, d_out);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_ray_vjp(const double* d_rbar, int32_t n_nodes, const int32_t* d_node_ptr, const int32_t* d_node_row,
                    const double* d_node_val, const int32_t* d_nodes, double rho_l, double rho_g, int32_t nz,
                    int32_t nr, double* d_lam, void* hip_stream) {
    if (!d_rbar || !d_node_ptr || !d_node_row || !d_node_val || !d_nodes || !d_lam || n_nodes < 0 || rho_l == rho_g)
        return LBM_AXI_EINVAL;
    if (n_nodes == 0) return LBM_AXI_OK;
    hipLaunchKernelGGL(ray_vjp_kernel, dim3((n_nodes + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       d_rbar, d_node_ptr, d_node_row, d_node_val, d_nodes, n_nodes, rho_l, rho_g,
                       (long long)nz * nr, d_lam);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_misfit(const double* d_r, const double* d_target, int32_t m, double* d_loss, double* d_rbar,
                   void* hip_stream) {
    if (!d_r || !d_target || !d_loss || m < 0) return LBM_AXI_EINVAL;
    hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_r, d_target, m,
                       d_loss, d_rbar);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EHIP;
}

int lbm_axi_ray_weights(int32_t nz, int32_t nr, double zc, const double* h_thetas, int32_t n_rays, double ds,
                        double s_max, int32_t cap, int32_t* h_row_ptr, int32_t* h_col, double* h_val,
                        int32_t* h_node_ptr, int32_t* h_nodes, int32_t* h_node_row, double* h_node_val,
                        int32_t* h_nnz, int32_t* h_n_nodes) {
    if (nz < 1 || nr < 1 || n_rays < 0 || !(ds > 0.0) || !h_nnz || !h_n_nodes || (n_rays > 0 && !h_thetas))
        return LBM_AXI_EINVAL;
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
    int32_t nnz = 0;
    for (int m = 0; m < n_rays; ++m) {
        nnz += (int32_t)rows[m].size();
        for (const auto& kv : rows[m]) by_node[kv.first].push_back({m, kv.second});
    }
    *h_nnz = nnz;
    *h_n_nodes = (int32_t)by_node.size();
    if (!h_row_ptr || !h_col || !h_val || !h_node_ptr || !h_nodes || !h_node_row || !h_node_val) return LBM_AXI_OK;
    if (cap < nnz) return LBM_AXI_ENOMEM;
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
}

}  // extern "C"
