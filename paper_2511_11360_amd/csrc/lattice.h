// Velocity sets of the GPU path (its own tables, compile-time only).
//
// c_s^2 = 1/3 on every lattice (Sec. IV of the paper). D2Q9 for the 2-D
// hydrodynamics (Sec. III), D3Q19 or D3Q27 (the paper's own 3-D lattice) for
// the 3-D hydrodynamics, D2Q5 and D3Q7 for the phase field; with c_s^2 = 1/3
// the D3Q7 rest weight is 0.
// The population order is the canonical order of the C ABI (pflbm.h).
#pragma once

#include <type_traits>
#include <utility>

namespace pfk {

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1, so
// every table lookup below folds to an immediate.
template <class F, int... I>
__host__ __device__ __forceinline__ void unroll_seq(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void unroll(F&& f) {
    unroll_seq(f, std::make_integer_sequence<int, N>{});
}

struct D2Q9 {
    static constexpr int Q = 9;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
        return t[i][a];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int i) {
        constexpr int t[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        return t[i];
    }
    // first member of each opposite pair
    static constexpr int NP = 4;
    __host__ __device__ static constexpr int pf(int k) {
        constexpr int t[4] = {1, 2, 5, 6};
        return t[k];
    }
};

struct D2Q5 {
    static constexpr int Q = 5;
    __host__ __device__ static constexpr int c(int i, int a) { return D2Q9::c(i, a); }
    __host__ __device__ static constexpr double w(int i) { return i == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr int opp(int i) { return D2Q9::opp(i); }
    static constexpr int NP = 2;
    __host__ __device__ static constexpr int pf(int k) { return k + 1; }
};

struct D3Q19 {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[19][3] = {{0, 0, 0},
                                  {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
                                  {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
                                  {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                  {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        return t[i][a];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int i) {
        return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1);
    }
    static constexpr int NP = 9;
    __host__ __device__ static constexpr int pf(int k) { return 2 * k + 1; }
};

struct D3Q27 {
    static constexpr int Q = 27;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[8][3] = {{1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
                                 {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
        return i < 19 ? D3Q19::c(i, a) : t[i - 19][a];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 8.0 / 27.0 : (i < 7 ? 2.0 / 27.0 : (i < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
    }
    __host__ __device__ static constexpr int opp(int i) {
        return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1);
    }
    static constexpr int NP = 13;
    __host__ __device__ static constexpr int pf(int k) { return 2 * k + 1; }
};

// Squared norms (sum over the velocities) of the stress rows of the moment
// basis: 3 c_x^2 - c^2 and c_y^2 - c_z^2 in 3-D, c_x^2 - c_y^2 in 2-D, and
// c_x c_y (the same for the other off-diagonal rows by symmetry).
template <class L, int DIM>
__host__ __device__ constexpr double stress_norm_diag0() {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) {
        const int x2 = L::c(i, 0) * L::c(i, 0), y2 = L::c(i, 1) * L::c(i, 1), z2 = L::c(i, 2) * L::c(i, 2);
        const int v = DIM == 2 ? x2 - y2 : 3 * x2 - (x2 + y2 + z2);
        s += (double)(v * v);
    }
    return s;
}
template <class L>
__host__ __device__ constexpr double stress_norm_diag1() {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) {
        const int v = L::c(i, 1) * L::c(i, 1) - L::c(i, 2) * L::c(i, 2);
        s += (double)(v * v);
    }
    return s;
}
template <class L>
__host__ __device__ constexpr double stress_norm_off() {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) {
        const int v = L::c(i, 0) * L::c(i, 1);
        s += (double)(v * v);
    }
    return s;
}
// Their inverses as compile-time constants: the norm functions loop over the
// velocity table, and used in ordinary expressions they are not always folded
// (on D3Q27 the loop stayed in the kernel, run for every plane).
template <class L, int DIM>
struct StressNorms {
    static constexpr double inv_d0 = 1.0 / stress_norm_diag0<L, DIM>();
    static constexpr double inv_d1 = 1.0 / stress_norm_diag1<L>();
    static constexpr double inv_off = 1.0 / stress_norm_off<L>();
};
static_assert(stress_norm_diag0<D3Q19, 3>() == 36.0 && stress_norm_diag1<D3Q19>() == 12.0 &&
              stress_norm_off<D3Q19>() == 4.0, "D3Q19 stress norms");
static_assert(stress_norm_off<D3Q27>() == 12.0, "D3Q27 stress norm");
static_assert(stress_norm_diag0<D2Q9, 2>() == 4.0 && stress_norm_off<D2Q9>() == 4.0, "D2Q9 stress norms");

struct D3Q7 {
    static constexpr int Q = 7;
    __host__ __device__ static constexpr int c(int i, int a) { return D3Q19::c(i, a); }
    __host__ __device__ static constexpr double w(int i) { return i == 0 ? 0.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr int opp(int i) { return D3Q19::opp(i); }
    static constexpr int NP = 3;
    __host__ __device__ static constexpr int pf(int k) { return 2 * k + 1; }
};

// lattice pairs: G = hydrodynamic (also the finite-difference stencil), H = phase field
struct Pair2D {
    using G = D2Q9;
    using H = D2Q5;
    static constexpr int dim = 2;
};
struct Pair3D {
    using G = D3Q19;
    using H = D3Q7;
    static constexpr int dim = 3;
};
struct Pair3D27 {
    using G = D3Q27;
    using H = D3Q7;
    static constexpr int dim = 3;
};

}  // namespace pfk
