// D3Q39 lattice constants and compile-time unrolled sums for the device code.
//
// Velocity set: Sec. 3 of the paper (the E_{3,7}^{39} lattice): (0,0,0),
// (1,0,0)_FS, (+-1,+-1,+-1), (2,0,0)_FS, (2,2,0)_FS, (3,0,0)_FS.  Stored as
// the rest velocity followed by 19 opposite pairs: velocity 2p+1 is the
// representative c_p of pair p and velocity 2p+2 = -c_p.  Every sum over the
// 39 velocities is then written over the 19 pairs, with the pair sum
// s_p = h(c_p) + h(-c_p) for functions even in xi and the pair difference
// a_p = h(c_p) - h(-c_p) for odd ones, which halves the arithmetic.
//
// The 13 basis functions of the exponent (Eq. eq:discrete-equilibrium):
//   0: 1           1-3: xi_x, xi_y, xi_z           4-6: xi_x^2, xi_y^2, xi_z^2
//   7-9: xi_x xi_y, xi_x xi_z, xi_y xi_z           10-12: xi_a |xi|^2
// Even (unchanged by xi -> -xi): 0, 4..9.  Odd: 1..3, 10..12.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace lbm13 {

constexpr int kQ = 39;
constexpr int kPairs = 19;
constexpr int kM = 13;

// representatives of the 19 pairs, in pair order
constexpr int kPairVel[kPairs][3] = {
    {1, 0, 0},  {0, 1, 0},  {0, 0, 1},                                  // (1,0,0)_FS
    {1, 1, 1},  {1, 1, -1}, {1, -1, 1}, {-1, 1, 1},                     // (+-1,+-1,+-1)
    {2, 0, 0},  {0, 2, 0},  {0, 0, 2},                                  // (2,0,0)_FS
    {2, 2, 0},  {2, -2, 0}, {2, 0, 2},  {2, 0, -2}, {0, 2, 2}, {0, 2, -2},  // (2,2,0)_FS
    {3, 0, 0},  {0, 3, 0},  {0, 0, 3},                                  // (3,0,0)_FS
};

__host__ __device__ constexpr int vel(int i, int a)
{
    return i == 0 ? 0 : (((i - 1) & 1) == 0 ? kPairVel[(i - 1) >> 1][a] : -kPairVel[(i - 1) >> 1][a]);
}

__host__ __device__ constexpr int opposite(int i) { return i == 0 ? 0 : (((i - 1) & 1) == 0 ? i + 1 : i - 1); }

__host__ __device__ constexpr int pair_q(int p)
{
    return kPairVel[p][0] * kPairVel[p][0] + kPairVel[p][1] * kPairVel[p][1] + kPairVel[p][2] * kPairVel[p][2];
}

// basis function k evaluated at the representative of pair p
__host__ __device__ constexpr int phi_pair(int k, int p)
{
    const int x = kPairVel[p][0], y = kPairVel[p][1], z = kPairVel[p][2];
    const int q = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x;
    case 5: return y * y;
    case 6: return z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * q;
    case 11: return y * q;
    case 12: return z * q;
    }
    return 0;
}

// index 0..5 of the velocity shell |xi|^2 in {0, 1, 3, 4, 8, 9}
__host__ __device__ constexpr int shell_of_q(int q)
{
    return q == 0 ? 0 : q == 1 ? 1 : q == 3 ? 2 : q == 4 ? 3 : q == 8 ? 4 : 5;
}
__host__ __device__ constexpr int shell(int i)
{
    return shell_of_q(vel(i, 0) * vel(i, 0) + vel(i, 1) * vel(i, 1) + vel(i, 2) * vel(i, 2));
}

__host__ __device__ constexpr bool basis_odd(int k) { return (k >= 1 && k <= 3) || k >= 10; }

// acc + c * v with the constant c folded at compile time (0: nothing,
// +-1: add/subtract, otherwise one multiply-add)
template <int c>
struct Term {
    template <class T>
    static __device__ __forceinline__ T add(T acc, T v) { return acc + T(c) * v; }
};
template <>
struct Term<0> {
    template <class T>
    static __device__ __forceinline__ T add(T acc, T) { return acc; }
};
template <>
struct Term<1> {
    template <class T>
    static __device__ __forceinline__ T add(T acc, T v) { return acc + v; }
};
template <>
struct Term<-1> {
    template <class T>
    static __device__ __forceinline__ T add(T acc, T v) { return acc - v; }
};

// sum_p phi_K(c_p) * v[p]
template <int K, class T, int... P>
__device__ __forceinline__ T basis_sum(const T *v, std::integer_sequence<int, P...>)
{
    T acc = T(-0.0);  // -0 + v folds to v
    ((acc = Term<phi_pair(K, P)>::add(acc, v[P])), ...);
    return acc;
}

// sum_p phi_K(c_p) phi_L(c_p) * v[p]
template <int K, int L, class T, int... P>
__device__ __forceinline__ T gram_sum(const T *v, std::integer_sequence<int, P...>)
{
    T acc = T(-0.0);  // -0 + v folds to v
    ((acc = Term<phi_pair(K, P) * phi_pair(L, P)>::add(acc, v[P])), ...);
    return acc;
}

// phi_K(c_p) . lam restricted to even (Odd = false) or odd basis functions
template <bool Odd, int P, class T, int... K>
__device__ __forceinline__ T exponent_part(const T *lam, std::integer_sequence<int, K...>)
{
    T acc = T(-0.0);  // -0 + v folds to v
    ((acc = (basis_odd(K) == Odd) ? Term<phi_pair(K, P)>::add(acc, lam[K]) : acc), ...);
    return acc;
}

using PairSeq = std::make_integer_sequence<int, kPairs>;
using BasisSeq = std::make_integer_sequence<int, kM>;

}  // namespace lbm13
