// D2Q9 lattice of the axisymmetric Shan–Chen scheme, as compile-time
// functions usable in device code after loop unrolling.
//
// Velocities are (c_z, c_r): direction 0 is at rest, 1..4 are the axial and
// radial links c_1 = +z, c_2 = +r, c_3 = -z, c_4 = -r (the assignment the
// mixed-derivative stencil of Sec. II.D needs), 5..8 the diagonals.
// Weights 4/9, 1/9, 1/36 and c_s^2 = 1/3 (appendix, Eq. e_distribution).
#pragma once

namespace lbm {

constexpr int kQ = 9;

__host__ __device__ constexpr int cz(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}

__host__ __device__ constexpr int cr(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}

__host__ __device__ constexpr double weight(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

// direction with velocity (c_z, -c_r): specular reflection at a plane r = const
__host__ __device__ constexpr int mirror_r(int i) {
    return i == 2 ? 4 : i == 4 ? 2 : i == 5 ? 8 : i == 8 ? 5 : i == 6 ? 7 : i == 7 ? 6 : i;
}

// direction with velocity -c: bounce-back
__host__ __device__ constexpr int opposite(int i) {
    return i == 0 ? 0 : i == 1 ? 3 : i == 3 ? 1 : i == 2 ? 4 : i == 4 ? 2 : i == 5 ? 7 : i == 7 ? 5 : i == 6 ? 8 : 6;
}

}  // namespace lbm
