// Device arithmetic of the 13-moment exponential equilibrium (Sec. 2 of the
// paper, Eq. eq:discrete-equilibrium) and its Newton-Raphson solve (Sec. 3 and
// the algorithm table of Sec. 5), templated on the arithmetic type C (double
// or float).  Everything is written per lane (one cell per lane) with all
// loops unrolled at compile time so that the lattice constants fold into the
// instruction stream.
#pragma once

#include "d3q39.h"
#include "slot.h"

namespace lbm13 {

template <class C>
__device__ __forceinline__ C dexp(C x);

// exp in FP64 by Cody and Waite's argument reduction, x = k ln2 + r with
// |r| <= ln2 / 2 (ln2 split into a 32-bit head, exact in k * head, and a
// tail), and the degree-10 polynomial of least maximum relative error for
// e^r on that interval (Remez exchange; relative error 2.1e-16 before
// rounding; coefficients from exp_minimax.py in the package), scaled by 2^k.
// Non-finite or out-of-range arguments give non-finite or zero results
// through the scaling, which the solver treats as a failed evaluation.
template <>
__device__ __forceinline__ double dexp<double>(double x)
{
    constexpr double kLog2e = 0x1.71547652b82fep+0;
    constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
    constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
    const double k = __builtin_rint(x * kLog2e);
    double r = __builtin_fma(-k, kLn2Hi, x);
    r = __builtin_fma(-k, kLn2Lo, r);
    double p = 0x1.2727a88044faap-22;
    p = __builtin_fma(p, r, 0x1.72f98543deccbp-19);
    p = __builtin_fma(p, r, 0x1.a01b6ce393267p-16);
    p = __builtin_fma(p, r, 0x1.a0197a4e9bd9dp-13);
    p = __builtin_fma(p, r, 0x1.6c16c0c0acbd4p-10);
    p = __builtin_fma(p, r, 0x1.1111112d4977ep-7);
    p = __builtin_fma(p, r, 0x1.55555555933c2p-5);
    p = __builtin_fma(p, r, 0x1.555555554bc09p-3);
    p = __builtin_fma(p, r, 0x1.ffffffffffe17p-2);
    p = __builtin_fma(p, r, 0x1.000000000001dp+0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(p, (int)k);
}
template <>
__device__ __forceinline__ float dexp<float>(float x) { return __expf(x); }  // v_exp_f32 on x log2(e)

template <class C>
__device__ __forceinline__ C dlog(C x);
template <>
__device__ __forceinline__ double dlog<double>(double x) { return log(x); }
template <>
__device__ __forceinline__ float dlog<float>(float x) { return logf(x); }

template <class C>
__device__ __forceinline__ C dsqrt(C x);
template <>
__device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }
template <>
__device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }

// 1/sqrt(x) and 1/x: exact division in FP64; the hardware approximations
// (about 1 ulp) in the FP32 path.
// FP64: the hardware estimates refined by two Newton steps each (each step
// squares the relative error), in place of the full-precision division and
// square-root sequences; used for the Cholesky pivots and the sensor, whose
// results need accuracy to a few ulp, not correct rounding
__device__ __forceinline__ double rsqrt_(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-(x * y), y, 1.0);  // 1 - x y^2
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-(x * y), y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);  // 1 - x y
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Maxwell-Boltzmann targets per unit density (Eq. eq:EqMomentsTensor, the 13
// constraints of Eq. eq:13constraints; the contracted third moment is
// u_a (|u|^2 + (D + 2) T) with D = 3).
template <class C>
__device__ __forceinline__ void mb_targets(const C u[3], C T, C m[kM])
{
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const C h = uu + C(5) * T;
    m[0] = C(1);
    m[1] = u[0];
    m[2] = u[1];
    m[3] = u[2];
    m[4] = u[0] * u[0] + T;
    m[5] = u[1] * u[1] + T;
    m[6] = u[2] * u[2] + T;
    m[7] = u[0] * u[1];
    m[8] = u[0] * u[2];
    m[9] = u[1] * u[2];
    m[10] = h * u[0];
    m[11] = h * u[1];
    m[12] = h * u[2];
}

// exp(phi_i . lam) for the rest velocity (f0) and both members of every pair
template <int P, class C>
__device__ __forceinline__ void eval_pair(const C *lam, C *fp, C *fm)
{
    const C e = exponent_part<false, P>(lam, BasisSeq{});
    const C o = exponent_part<true, P>(lam, BasisSeq{});
    fp[P] = dexp(e + o);
    fm[P] = dexp(e - o);
}

template <class C, int... P>
__device__ __forceinline__ void eval_pairs(const C *lam, C *fp, C *fm, std::integer_sequence<int, P...>)
{
    (eval_pair<P>(lam, fp, fm), ...);
}

template <class C>
__device__ __forceinline__ void eval_exponentials(const C lam[kM], C &f0, C fp[kPairs], C fm[kPairs])
{
    f0 = dexp(lam[0]);
    eval_pairs(lam, fp, fm, PairSeq{});
}

// Target k of mb_targets evaluated from (u, T, h = |u|^2 + 5T)
template <int K, class C>
__device__ __forceinline__ C target(const C u[3], C T, C h)
{
    if constexpr (K == 0) return C(1);
    else if constexpr (K <= 3) return u[K - 1];
    else if constexpr (K <= 6) return u[K - 4] * u[K - 4] + T;
    else if constexpr (K == 7) return u[0] * u[1];
    else if constexpr (K == 8) return u[0] * u[2];
    else if constexpr (K == 9) return u[1] * u[2];
    else return h * u[K - 10];
}

// G_k = sum_i exp(phi_i . lam) phi_ik - m_k from pair sums s and differences a
template <class C, int... K>
__device__ __forceinline__ void residual_impl(C f0, const C *s, const C *a, const C u[3], C T, C h, C *G,
                                              std::integer_sequence<int, K...>)
{
    ((G[K] = ((K == 0) ? f0 : C(-0.0)) + basis_sum<K>(basis_odd(K) ? a : s, PairSeq{}) - target<K>(u, T, h)), ...);
}

template <int K, int L, class C>
__device__ __forceinline__ C jac_entry(C f0, const C *s, const C *a)
{
    constexpr bool odd = basis_odd(K) != basis_odd(L);
    C v = gram_sum<K, L>(odd ? a : s, PairSeq{});
    if constexpr (K == 0 && L == 0) v = f0 + v;
    return v;
}

template <int L, class C, int... K>
__device__ __forceinline__ void jac_row(C f0, const C *s, const C *a, C (&J)[kM][kM], std::integer_sequence<int, K...>)
{
    ((J[L][K] = jac_entry<K, L>(f0, s, a)), ...);
}

// lower triangle of J_kl = sum_i exp(phi_i . lam) phi_ik phi_il
template <class C, int... L>
__device__ __forceinline__ void jacobian_impl(C f0, const C *s, const C *a, C (&J)[kM][kM],
                                              std::integer_sequence<int, L...>)
{
    (jac_row<L>(f0, s, a, J, std::make_integer_sequence<int, L + 1>{}), ...);
}

// Solve J d = G.  The paper inverts J; J is symmetric positive definite, so
// a Cholesky factorisation gives the same d.  Returns false if a pivot is not
// positive (or not a number).
template <class C>
__device__ __forceinline__ bool cholesky_solve(C (&J)[kM][kM], const C G[kM], C d[kM])
{
    bool ok = true;
    C rdiag[kM];
#pragma unroll
    for (int j = 0; j < kM; ++j) {
        C s = J[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= J[j][k] * J[j][k];
        ok = ok && (s > C(0));
        const C r = rsqrt_(s);
        rdiag[j] = r;
#pragma unroll
        for (int i = j + 1; i < kM; ++i) {
            C t = J[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= J[i][k] * J[j][k];
            J[i][j] = t * r;
        }
    }
    C y[kM];
#pragma unroll
    for (int i = 0; i < kM; ++i) {
        C t = G[i];
#pragma unroll
        for (int k = 0; k < i; ++k) t -= J[i][k] * y[k];
        y[i] = t * rdiag[i];
    }
#pragma unroll
    for (int i = kM - 1; i >= 0; --i) {
        C t = y[i];
#pragma unroll
        for (int k = i + 1; k < kM; ++k) t -= J[k][i] * d[k];
        d[i] = t * rdiag[i];
    }
    return ok;
}

// Multipliers of the Maxwellian shape (cold start): lam_1 = u/T,
// lam_2 = -delta/(2T), lam_3 = 0; lam_0 is set by the solver so that the
// exponentials sum to 1.
template <class C>
__device__ __forceinline__ void maxwellian_shape(const C u[3], C T, C lam[kM])
{
#pragma unroll
    for (int k = 0; k < kM; ++k) lam[k] = C(0);
    lam[1] = u[0] / T;
    lam[2] = u[1] / T;
    lam[3] = u[2] / T;
    lam[4] = lam[5] = lam[6] = C(-0.5) / T;
}

// lam_0 = -log of the sum of the exponentials at lam_0 = 0, so that the
// exponentials sum to 1
template <class C>
__device__ __forceinline__ void normalise_lam0(C lam[kM])
{
    lam[0] = C(0);
    C f0, fp[kPairs], fm[kPairs];
    eval_exponentials(lam, f0, fp, fm);
    C sum = f0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) sum += fp[p] + fm[p];
    lam[0] = -dlog(sum);
}

// how solve_multipliers starts
enum SolveStart : int {
    kStartWarm = 0,    // from lam; one cold restart if that fails
    kStartMarked = 1,  // from lam_1..12 of a cell that failed the previous step (lam_0 not valid); no cold restart
    kStartCold = 2,    // from the Maxwellian shape only
};

// Newton-Raphson for the multipliers, warm-started from lam.  Stopping rule:
// max_k |G_k| <= tol * max(1, max_k |m_k|).  Step halving while the Euclidean
// norm of G does not decrease, trying t = 1, 1/2, ..., 2^-39; when no trial
// lowers it the attempt has stalled and fails (no descent is left, which is
// what happens where no multipliers satisfy the constraints).  If the warm
// start fails (cap reached, stall, J not positive definite, or a value not
// finite) the solve restarts once from the Maxwellian shape with cap
// maxit_cold (start = kStartWarm only).  Where lam_0 is to be set (kStartMarked
// and every cold start) it is -log of the sum of the exponentials at
// lam_0 = 0, so that the start sums to 1.  On return lam, f0, fp, fm
// hold the last accepted iterate, G its residual (all zero after a failure),
// and iters the number of accepted updates of the final attempt (maxit if the
// solve failed).  The targets m are evaluated from (u, T) where needed.
template <class C>
__device__ __forceinline__ int solve_multipliers(const C u[3], C T, C lam[kM], C &f0, C fp[kPairs], C fm[kPairs],
                                                 C tol, int maxit, int maxit_cold, int start, int &iters,
                                                 C (&G)[kM])
{
    C m[kM];
    mb_targets(u, T, m);
    C scale = C(1);
#pragma unroll
    for (int k = 0; k < kM; ++k) scale = fabs(m[k]) > scale ? fabs(m[k]) : scale;
    const C bound = tol * scale;
    const C h = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + C(5) * T;

    // lam holds the trial point lam_acc - t d; a rejected trial moves back by
    // half its step (t -> t/2)
    C d[kM];
#pragma unroll
    for (int k = 0; k < kM; ++k) d[k] = C(0);
    C t = C(0);
    C n0 = C(0);
    const bool from_cold = start == kStartCold;
    int it = 0, ls = 0, cap = from_cold ? maxit_cold : maxit;
    bool fresh = true, cold = start != kStartWarm, floor_stop = false;
    bool restarted = from_cold;  // the current attempt started from the Maxwellian shape
    bool near = false;  // the last accepted iterate is within 8 times the bound
    int status = kFailed;
    if (from_cold) maxwellian_shape(u, T, lam);
    if (start != kStartWarm) normalise_lam0(lam);
    for (;;) {
        eval_exponentials(lam, f0, fp, fm);
        C s[kPairs], a[kPairs];
#pragma unroll
        for (int p = 0; p < kPairs; ++p) {
            s[p] = fp[p] + fm[p];
            a[p] = fp[p] - fm[p];
        }
        residual_impl(f0, s, a, u, T, h, G, BasisSeq{});
        C n2 = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) n2 += G[k] * G[k];
        n2 = dsqrt(n2);
        C r = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const C g = fabs(G[k]);
            r = (g <= r) ? r : g;  // NaN propagates
        }
        // the full step does not lower the residual, but the accepted iterate
        // and the step's end are both within 8 times the bound: the residual
        // sits at the round-off floor; the step is taken and the solve stops
        floor_stop = !fresh && !(n2 < n0) && ls == 0 && near && r <= C(8) * bound;
        const bool rejected = !fresh && !(n2 < n0) && !floor_stop;
        if (rejected && ls < 39) {
            t *= C(0.5);
            ++ls;
#pragma unroll
            for (int k = 0; k < kM; ++k) lam[k] += t * d[k];
            continue;
        }
        bool bad = rejected;  // no trial lowered the residual: stalled
        if (!bad) {
            if (!fresh) ++it;
            fresh = false;
            near = r <= C(8) * bound;
            if (r <= bound || floor_stop) {
                status = restarted ? kConvergedCold : kConverged;
                break;
            }
            bad = !(r - r == C(0)) || it >= cap;  // not finite, or cap reached
        }
        if (!bad) {
            C J[kM][kM];
            jacobian_impl(f0, s, a, J, BasisSeq{});
            bad = !cholesky_solve(J, G, d);
        }
        if (bad) {
            if (cold) {
                status = kFailed;
                break;
            }
            cold = true;
            restarted = true;
            maxwellian_shape(u, T, lam);
            normalise_lam0(lam);
            it = 0;
            ls = 0;
            cap = maxit_cold;
            fresh = true;
            continue;
        }
        t = C(1);
        ls = 0;
        n0 = n2;
#pragma unroll
        for (int k = 0; k < kM; ++k) lam[k] -= d[k];
    }
    if (status == kFailed) {
        // no equilibrium: leave finite values behind (the caller does not
        // relax such a cell, and omega = 0 times a finite difference is 0);
        // zero residuals keep the invariant projection a no-op
        f0 = C(0);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) fp[p] = fm[p] = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) G[k] = C(0);
    }
    iters = status == kFailed ? maxit : it;
    return status;
}

// ---------------------------------------------------------------------------
// Secant variant of the root finder (Sec. 6 leaves the choice between
// gradient-based and gradient-free algorithms open): the Jacobian of G is
// never evaluated.  G is the gradient of the convex dual
// Phi(lam) = sum_i exp(phi_i . lam) - lam . m, and limited-memory BFGS builds
// the inverse Jacobian from the steps s and residual changes y of the last
// kSecantMemory accepted updates, on top of a model inverse H0.

constexpr int kSecantMemory = 3;

// r = H0 v with H0 the inverse of the model Jacobian A(u) D J_rest D A(u)^T:
// J_rest is the Jacobian of the rest equilibrium at T_ref, D = diag(s^-deg_k)
// with s = sqrt(T_ref / T) and deg_k the degree of basis function k in xi,
// and A(w) the shift of the basis, phi(xi + w) = A(w) phi(xi) (the span of
// the 13 functions is closed under shifts).  Since A(u)^-1 = A(-u),
//     H0 = A(w)^T D^-1 H_rest D^-1 A(w),  w = -u,
// applied here factor by factor; H_rest = J_rest^-1 has the cubic-symmetric
// blocks of h (see SlotDesc::qn_h).  For the continuous Maxwellian this
// model is exact.
template <class C>
__device__ __forceinline__ void model_inverse_apply(const double (&h)[8], C sc, const C w[3], const C v[kM],
                                                    C r[kM])
{
    const C w0 = w[0], w1 = w[1], w2 = w[2];
    const C ww = w0 * w0 + w1 * w1 + w2 * w2;
    const C tr = v[4] + v[5] + v[6];
    C x[kM];
    // x = A(w) v
    x[0] = v[0];
    x[1] = w0 * v[0] + v[1];
    x[2] = w1 * v[0] + v[2];
    x[3] = w2 * v[0] + v[3];
    x[4] = w0 * w0 * v[0] + C(2) * w0 * v[1] + v[4];
    x[5] = w1 * w1 * v[0] + C(2) * w1 * v[2] + v[5];
    x[6] = w2 * w2 * v[0] + C(2) * w2 * v[3] + v[6];
    x[7] = w0 * w1 * v[0] + w1 * v[1] + w0 * v[2] + v[7];
    x[8] = w0 * w2 * v[0] + w2 * v[1] + w0 * v[3] + v[8];
    x[9] = w1 * w2 * v[0] + w2 * v[2] + w1 * v[3] + v[9];
    x[10] = ww * w0 * v[0] + (C(2) * w0 * w0 + ww) * v[1] + C(2) * w0 * w1 * v[2] + C(2) * w0 * w2 * v[3] +
            w0 * tr + C(2) * w0 * v[4] + C(2) * w1 * v[7] + C(2) * w2 * v[8] + v[10];
    x[11] = ww * w1 * v[0] + C(2) * w1 * w0 * v[1] + (C(2) * w1 * w1 + ww) * v[2] + C(2) * w1 * w2 * v[3] +
            w1 * tr + C(2) * w1 * v[5] + C(2) * w0 * v[7] + C(2) * w2 * v[9] + v[11];
    x[12] = ww * w2 * v[0] + C(2) * w2 * w0 * v[1] + C(2) * w2 * w1 * v[2] + (C(2) * w2 * w2 + ww) * v[3] +
            w2 * tr + C(2) * w2 * v[6] + C(2) * w0 * v[8] + C(2) * w1 * v[9] + v[12];
    // D^-1, H_rest, D^-1
    const C s1 = sc, s2 = sc * sc, s3 = s2 * sc;
#pragma unroll
    for (int k = 1; k <= 3; ++k) x[k] *= s1;
#pragma unroll
    for (int k = 4; k <= 9; ++k) x[k] *= s2;
#pragma unroll
    for (int k = 10; k <= 12; ++k) x[k] *= s3;
    C y[kM];
    const C h00 = C(h[0]), h0s = C(h[1]), hss = C(h[2]), hst = C(h[3]);
    const C h11 = C(h[4]), h1q = C(h[5]), hqq = C(h[6]), hp = C(h[7]);
    const C S = x[4] + x[5] + x[6];
    y[0] = h00 * x[0] + h0s * S;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        y[4 + a] = h0s * x[0] + (hss - hst) * x[4 + a] + hst * S;
        y[1 + a] = h11 * x[1 + a] + h1q * x[10 + a];
        y[10 + a] = h1q * x[1 + a] + hqq * x[10 + a];
        y[7 + a] = hp * x[7 + a];
    }
#pragma unroll
    for (int k = 1; k <= 3; ++k) y[k] *= s1;
#pragma unroll
    for (int k = 4; k <= 9; ++k) y[k] *= s2;
#pragma unroll
    for (int k = 10; k <= 12; ++k) y[k] *= s3;
    // r = A(w)^T y
    const C wq = w0 * y[10] + w1 * y[11] + w2 * y[12];
    r[0] = y[0] + w0 * y[1] + w1 * y[2] + w2 * y[3] + w0 * w0 * y[4] + w1 * w1 * y[5] + w2 * w2 * y[6] +
           w0 * w1 * y[7] + w0 * w2 * y[8] + w1 * w2 * y[9] + ww * wq;
    r[1] = y[1] + C(2) * w0 * y[4] + w1 * y[7] + w2 * y[8] + ww * y[10] + C(2) * w0 * wq;
    r[2] = y[2] + C(2) * w1 * y[5] + w0 * y[7] + w2 * y[9] + ww * y[11] + C(2) * w1 * wq;
    r[3] = y[3] + C(2) * w2 * y[6] + w0 * y[8] + w1 * y[9] + ww * y[12] + C(2) * w2 * wq;
    r[4] = y[4] + wq + C(2) * w0 * y[10];
    r[5] = y[5] + wq + C(2) * w1 * y[11];
    r[6] = y[6] + wq + C(2) * w2 * y[12];
    r[7] = y[7] + C(2) * w1 * y[10] + C(2) * w0 * y[11];
    r[8] = y[8] + C(2) * w2 * y[10] + C(2) * w0 * y[12];
    r[9] = y[9] + C(2) * w2 * y[11] + C(2) * w1 * y[12];
    r[10] = y[10];
    r[11] = y[11];
    r[12] = y[12];
}

// The secant variant of solve_multipliers (same arguments, starts, stopping
// rule, round-off floor stop, stall, cold restart and outputs; iters counts
// accepted updates).  Direction d = H G by the two-loop recursion over the
// stored pairs (s = -t d, the step taken, and y = G_new - G_old, kept only
// when s . y > 0, the oldest dropped beyond kSecantMemory) on H0 =
// model_inverse_apply; trial lam - t d, t = 1, 1/2, ..., 2^-39.  A trial is
// accepted when it lowers ||G||_2, or, for a descent direction (G . d > 0),
// when it lowers Phi by at least 1e-4 t G . d (Armijo on the dual, which a
// positive definite H guarantees for small t).  A cold restart drops the
// stored pairs.
template <class C>
__device__ __forceinline__ int solve_multipliers_secant(const C u[3], C T, C lam[kM], C &f0, C fp[kPairs],
                                                        C fm[kPairs], C tol, int maxit, int maxit_cold, int start,
                                                        int &iters, C (&G)[kM], const double (&hq)[8],
                                                        double T_ref)
{
    C m[kM];
    mb_targets(u, T, m);
    C scale = C(1);
#pragma unroll
    for (int k = 0; k < kM; ++k) scale = fabs(m[k]) > scale ? fabs(m[k]) : scale;
    const C bound = tol * scale;
    const C h = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + C(5) * T;
    const C w[3] = {-u[0], -u[1], -u[2]};
    const C sc = dsqrt(C(T_ref) / T);

    C Sp[kSecantMemory][kM], Yp[kSecantMemory][kM], rs[kSecantMemory];
#pragma unroll
    for (int j = 0; j < kSecantMemory; ++j) {
        rs[j] = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) Sp[j][k] = Yp[j][k] = C(0);
    }
    int np = 0;
    C Gacc[kM], d[kM];
#pragma unroll
    for (int k = 0; k < kM; ++k) Gacc[k] = d[k] = C(0);
    C t = C(0), n0 = C(0), phi0 = C(0), gd = C(0);
    const bool from_cold = start == kStartCold;
    int it = 0, ls = 0, cap = from_cold ? maxit_cold : maxit;
    bool fresh = true, cold = start != kStartWarm, floor_stop = false;
    bool restarted = from_cold;
    bool near = false;
    int status = kFailed;
    if (from_cold) maxwellian_shape(u, T, lam);
    if (start != kStartWarm) normalise_lam0(lam);
    for (;;) {
        eval_exponentials(lam, f0, fp, fm);
        {
            C s[kPairs], a[kPairs];
#pragma unroll
            for (int p = 0; p < kPairs; ++p) {
                s[p] = fp[p] + fm[p];
                a[p] = fp[p] - fm[p];
            }
            residual_impl(f0, s, a, u, T, h, G, BasisSeq{});
        }
        C n2 = C(0), lm = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            n2 += G[k] * G[k];
            lm += lam[k] * m[k];
        }
        n2 = dsqrt(n2);
        // dual objective: sum_i exp(phi_i . lam) - lam . m, the sum being G_0 + m_0
        const C phi = (G[0] + m[0]) - lm;
        C r = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const C g = fabs(G[k]);
            r = (g <= r) ? r : g;
        }
        const bool lower = (n2 < n0) || (gd > C(0) && phi <= phi0 - C(1e-4) * t * gd);
        floor_stop = !fresh && !lower && ls == 0 && near && r <= C(8) * bound;
        const bool rejected = !fresh && !lower && !floor_stop;
        if (rejected && ls < 39) {
            t *= C(0.5);
            ++ls;
#pragma unroll
            for (int k = 0; k < kM; ++k) lam[k] += t * d[k];
            continue;
        }
        bool bad = rejected;
        if (!bad) {
            if (!fresh) {
                ++it;
                C sy = C(0);
#pragma unroll
                for (int k = 0; k < kM; ++k) sy += (-t * d[k]) * (G[k] - Gacc[k]);
                if (sy > C(0)) {
#pragma unroll
                    for (int j = 0; j + 1 < kSecantMemory; ++j) {
                        rs[j] = rs[j + 1];
#pragma unroll
                        for (int k = 0; k < kM; ++k) {
                            Sp[j][k] = Sp[j + 1][k];
                            Yp[j][k] = Yp[j + 1][k];
                        }
                    }
                    rs[kSecantMemory - 1] = C(1) / sy;
#pragma unroll
                    for (int k = 0; k < kM; ++k) {
                        Sp[kSecantMemory - 1][k] = -t * d[k];
                        Yp[kSecantMemory - 1][k] = G[k] - Gacc[k];
                    }
                    np = np < kSecantMemory ? np + 1 : kSecantMemory;
                }
            }
            fresh = false;
            near = r <= C(8) * bound;
            if (r <= bound || floor_stop) {
                status = restarted ? kConvergedCold : kConverged;
                break;
            }
            bad = !(r - r == C(0)) || it >= cap;
        }
        if (!bad) {
            // two-loop recursion, newest pair first; pairs sit at the end
            C q[kM], al[kSecantMemory];
#pragma unroll
            for (int k = 0; k < kM; ++k) q[k] = G[k];
#pragma unroll
            for (int j = kSecantMemory - 1; j >= 0; --j) {
                C sq = C(0);
#pragma unroll
                for (int k = 0; k < kM; ++k) sq += Sp[j][k] * q[k];
                al[j] = j >= kSecantMemory - np ? rs[j] * sq : C(0);
#pragma unroll
                for (int k = 0; k < kM; ++k) q[k] -= al[j] * Yp[j][k];
            }
            model_inverse_apply(hq, sc, w, q, d);
#pragma unroll
            for (int j = 0; j < kSecantMemory; ++j) {
                C yd = C(0);
#pragma unroll
                for (int k = 0; k < kM; ++k) yd += Yp[j][k] * d[k];
                const C b = j >= kSecantMemory - np ? al[j] - rs[j] * yd : C(0);
#pragma unroll
                for (int k = 0; k < kM; ++k) d[k] += Sp[j][k] * b;
            }
            gd = C(0);
#pragma unroll
            for (int k = 0; k < kM; ++k) gd += G[k] * d[k];
            bad = !(gd - gd == C(0));
        }
        if (bad) {
            if (cold) {
                status = kFailed;
                break;
            }
            cold = true;
            restarted = true;
            maxwellian_shape(u, T, lam);
            normalise_lam0(lam);
            it = 0;
            ls = 0;
            cap = maxit_cold;
            fresh = true;
            np = 0;
            gd = C(0);
            continue;
        }
#pragma unroll
        for (int k = 0; k < kM; ++k) Gacc[k] = G[k];
        t = C(1);
        ls = 0;
        n0 = n2;
        phi0 = phi;
#pragma unroll
        for (int k = 0; k < kM; ++k) lam[k] -= d[k];
    }
    if (status == kFailed) {
        f0 = C(0);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) fp[p] = fm[p] = C(0);
#pragma unroll
        for (int k = 0; k < kM; ++k) G[k] = C(0);
    }
    iters = status == kFailed ? maxit : it;
    return status;
}

// Remove the residuals of the five collision invariants, R = sum_i f_i psi_i
// - target with psi = (1, xi, |xi|^2), that a solve stopped at a tolerance
// leaves in the equilibrium f (per unit density):
//     f_i <- f_i (1 + x . psi_i),   M x = -R,   M = sum_i f_i psi_i psi_i^T,
// after which sum_i f_i psi_i equals the targets exactly in exact
// arithmetic.  The correction of each population is proportional to the
// population itself, so it keeps every population's relative change at the
// level of the residuals, however small the population.  The entries of M
// are moments of f: the constrained ones are target + residual (the residual
// G of the accepted iterate), and sum_i f_i |xi_i|^4 is summed here.  M is a
// Gram matrix of 5 independent functions with positive weights, hence SPD;
// its Cholesky factor gives x.  ok = false (no equilibrium) leaves f alone.
template <class C>
__device__ __forceinline__ void project_invariants(C &f0, C *fp, C *fm, const C u[3], C T, const C (&G)[kM],
                                                   bool ok)
{
    C q4 = C(-0.0);
    [&]<int... P>(std::integer_sequence<int, P...>) {
        ((q4 = Term<pair_q(P) * pair_q(P)>::add(q4, fp[P] + fm[P])), ...);
    }(PairSeq{});
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const C h = uu + C(5) * T;
    // M in the order (1, xi_x, xi_y, xi_z, |xi|^2); lower triangle
    C M[5][5];
    M[0][0] = C(1) + G[0];
    M[1][0] = u[0] + G[1];
    M[2][0] = u[1] + G[2];
    M[3][0] = u[2] + G[3];
    M[4][0] = (uu + C(3) * T) + ((G[4] + G[5]) + G[6]);
    M[1][1] = u[0] * u[0] + T + G[4];
    M[2][2] = u[1] * u[1] + T + G[5];
    M[3][3] = u[2] * u[2] + T + G[6];
    M[2][1] = u[0] * u[1] + G[7];
    M[3][1] = u[0] * u[2] + G[8];
    M[3][2] = u[1] * u[2] + G[9];
    M[4][1] = h * u[0] + G[10];
    M[4][2] = h * u[1] + G[11];
    M[4][3] = h * u[2] + G[12];
    M[4][4] = q4;
    const C R[5] = {G[0], G[1], G[2], G[3], (G[4] + G[5]) + G[6]};
    // Cholesky M = L L^T in place (L scaled by the reciprocal pivots)
    C rd[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        C sj = M[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) sj -= M[j][k] * M[j][k];
        rd[j] = rsqrt_(sj);
#pragma unroll
        for (int i = j + 1; i < 5; ++i) {
            C tij = M[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) tij -= M[i][k] * M[j][k];
            M[i][j] = tij * rd[j];
        }
    }
    C y[5], x[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        C ti = -R[i];
#pragma unroll
        for (int k = 0; k < i; ++k) ti -= M[i][k] * y[k];
        y[i] = ti * rd[i];
    }
#pragma unroll
    for (int i = 4; i >= 0; --i) {
        C ti = y[i];
#pragma unroll
        for (int k = i + 1; k < 5; ++k) ti -= M[k][i] * x[k];
        x[i] = ti * rd[i];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) x[k] = ok ? x[k] : C(0);
    f0 += f0 * x[0];
    [&]<int... P>(std::integer_sequence<int, P...>) {
        (
            [&] {
                constexpr int cx = kPairVel[P][0], cy = kPairVel[P][1], cz = kPairVel[P][2];
                const C even = Term<pair_q(P)>::add(x[0], x[4]);
                C odd = C(-0.0);
                odd = Term<cx>::add(odd, x[1]);
                odd = Term<cy>::add(odd, x[2]);
                odd = Term<cz>::add(odd, x[3]);
                fp[P] += fp[P] * (even + odd);
                fm[P] += fm[P] * (even - odd);
            }(),
            ...);
    }(PairSeq{});
}

// equilibrium per unit density of velocity i from the solve's exponentials
template <int I, class C>
__device__ __forceinline__ C feq_of(C f0, const C *fp, const C *fm)
{
    if constexpr (I == 0) return f0;
    else if constexpr (((I - 1) & 1) == 0) return fp[(I - 1) >> 1];
    else return fm[(I - 1) >> 1];
}

}  // namespace lbm13
