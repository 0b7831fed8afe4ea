// lattice.hpp -- compile-time velocity sets in the interface order of lbm.h.
//
// D2Q9, D3Q19 and D3Q27 with c_s^2 = 1/3 (Sec. 2.2; the paper's 3D runs use
// D3Q27).  Every loop over populations
// in the kernels is unrolled with static_for, so each xi_i and w_i below is a
// literal in the generated code: no table is read at run time.
#pragma once

#include <type_traits>
#include <utility>

namespace lbm {

template <int Q>
struct Lattice;

template <>
struct Lattice<9> {
    static constexpr int D = 2;
    static constexpr int c[9][3] = {{0, 0, 0}, {1, 0, 0},  {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    // weights by squared length: 4/9, 1/9, 1/36
    static constexpr double w_by_len2[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
};

template <>
struct Lattice<19> {
    static constexpr int D = 3;
    static constexpr int c[19][3] = {
        {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
        {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
        {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    // weights by squared length: 1/3, 1/18, 1/36
    static constexpr double w_by_len2[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
};

template <>
struct Lattice<27> {
    static constexpr int D = 3;
    static constexpr int c[27][3] = {
        {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
        {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
        {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}, {1, 1, 1},   {-1, -1, -1},
        {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
    // weights by squared length: 8/27, 2/27, 1/54, 1/216
    static constexpr double w_by_len2[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
};

constexpr int kMaxQ = 27;

template <int Q, int I>
struct Vel {
    static constexpr int x = Lattice<Q>::c[I][0];
    static constexpr int y = Lattice<Q>::c[I][1];
    static constexpr int z = Lattice<Q>::c[I][2];
    static constexpr int len2 = x * x + y * y + z * z;
    static constexpr double w = Lattice<Q>::w_by_len2[len2];
    static constexpr int opp = (I == 0) ? 0 : ((I & 1) ? I + 1 : I - 1);
};

// Compile-time loop: f(std::integral_constant<int, I>{}) for I in [B, E).
template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(std::forward<F>(f));
    }
}

// Consistency of the table with its stated rules, checked at compile time.
template <int Q>
constexpr bool lattice_is_consistent() {
    for (int i = 0; i < Q; ++i) {
        const int o = (i == 0) ? 0 : ((i & 1) ? i + 1 : i - 1);
        for (int a = 0; a < 3; ++a)
            if (Lattice<Q>::c[o][a] != -Lattice<Q>::c[i][a]) return false;
    }
    return true;
}
static_assert(lattice_is_consistent<9>(), "D2Q9 opposite rule");
static_assert(lattice_is_consistent<19>(), "D3Q19 opposite rule");
static_assert(lattice_is_consistent<27>(), "D3Q27 opposite rule");

}  // namespace lbm
