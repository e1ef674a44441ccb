// Small dense algebra of the moment systems (App. B, eqs. A0, A1, A2_2),
// shared by the weight build and its adjoint so that both take the same
// arithmetic.
//
// Every system is the minimum-norm solution of M A = b, M the 6 x K matrix
// whose column k is the condition vector of support entry k.  Two solvers:
//  * the common one: A = M^t y, G y = b with G = M M^t formed from the 15
//    power sums of centred, scaled monomials, Cholesky with reciprocal
//    pivots, and a condition estimate trace(G) trace(G^-1) (within a factor
//    36 above cond2(G));
//  * the rank-revealing one, for systems whose estimate exceeds a threshold
//    or whose Cholesky breaks down: one-sided Jacobi on B = M^t, one support
//    entry per lane of a wave, singular values below eps max(6, K) s_max
//    dropped (App. A: SVD with automatic rank detection).
#pragma once

#include <cfloat>

#include "common.h"

namespace p2m {

constexpr double ALG_EPS = DBL_EPSILON;

__device__ __forceinline__ void monos(double x, double y, double p[6]) {
    p[0] = 1.0;
    p[1] = x;
    p[2] = y;
    p[3] = x * x;
    p[4] = x * y;
    p[5] = y * y;
}

__device__ __forceinline__ double dot6(const double a[6], const double b[6]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}

// The 15 power sums m_ab = sum x^a y^b (a + b <= 4).
struct Moments {
    double m[15];  // 00 10 01 20 11 02 30 21 12 03 40 31 22 13 04
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < 15; ++i) m[i] = 0.0;
    }
    __device__ void add(double x, double y) {
        const double x2 = x * x, y2 = y * y, xy = x * y;
        m[0] += 1.0;
        m[1] += x;
        m[2] += y;
        m[3] += x2;
        m[4] += xy;
        m[5] += y2;
        m[6] += x2 * x;
        m[7] += x2 * y;
        m[8] += x * y2;
        m[9] += y2 * y;
        m[10] += x2 * x2;
        m[11] += x2 * xy;
        m[12] += x2 * y2;
        m[13] += xy * y2;
        m[14] += y2 * y2;
    }
    // trace of the Gram matrix below
    __device__ double trace() const { return m[0] + m[3] + m[5] + m[10] + m[12] + m[14]; }
    // Gram matrix of p = (1, x, y, x^2, xy, y^2), lower triangle.
    __device__ void gram(double G[6][6]) const {
        G[0][0] = m[0];
        G[1][0] = m[1]; G[1][1] = m[3];
        G[2][0] = m[2]; G[2][1] = m[4]; G[2][2] = m[5];
        G[3][0] = m[3]; G[3][1] = m[6]; G[3][2] = m[7]; G[3][3] = m[10];
        G[4][0] = m[4]; G[4][1] = m[7]; G[4][2] = m[8]; G[4][3] = m[11]; G[4][4] = m[12];
        G[5][0] = m[5]; G[5][1] = m[8]; G[5][2] = m[9]; G[5][3] = m[12]; G[5][4] = m[13]; G[5][5] = m[14];
    }
};

// In-place Cholesky of the lower triangle; false if a pivot is not clearly
// positive (relative threshold on the squared pivot).  The diagonal keeps
// 1 / L_jj.
__device__ __forceinline__ bool chol6(double G[6][6]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double djj = G[j][j];
        double d = djj;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= G[j][k] * G[j][k];
        if (!(d > 1e-12 * djj)) return false;
        const double ir = 1.0 / sqrt(d);
        G[j][j] = ir;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = G[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= G[i][k] * G[j][k];
            G[i][j] = s * ir;
        }
    }
    return true;
}

__device__ __forceinline__ void chol6_solve(const double L[6][6], const double b[6], double y[6]) {
    double z[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
        z[i] = s * L[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = z[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[k][i] * y[k];
        y[i] = s * L[i][i];
    }
}

// trace(G^-1) = |L^-1|_F^2 from the factor of chol6, column by column.
// With trace(G) it brackets the condition number: cond2(G) <= trace(G)
// trace(G^-1) <= 36 cond2(G).
__device__ __forceinline__ double chol6_inv_trace(const double L[6][6]) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if (i < j) continue;
            double s = i == j ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k)
                if (k >= j) s -= L[i][k] * z[k];
            z[i] = s * L[i][i];
            t += z[i] * z[i];
        }
    }
    return t;
}

// ------------------------------------------------------ wave-wide helpers
// Sum over the 64 lanes by an xor butterfly: at every level a lane adds the
// partial of the group it meets, so every lane ends with the same bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ void wave_sum3(double& a, double& b, double& c) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        a += __shfl_xor(a, m, 64);
        b += __shfl_xor(b, m, 64);
        c += __shfl_xor(c, m, 64);
    }
}
// A value every lane holds with the same bits, read as a scalar so that the
// branches depending on it stay wave-uniform.
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(b));
    const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// ------------------------------------------- rank-revealing wave solver
// One-sided Jacobi on B = M^t (K x 6): lane k holds row k of B (the
// condition vector of support entry k; zero for lanes past the support),
// lanes 0..5 hold the rows of V.  Column pairs of B are rotated until every
// pair is orthogonal to working precision (or one of them is negligible);
// then B V has orthogonal columns of norms s_i, M = V S U^t, and the
// minimum-norm solution is A = sum over kept i of (B V)_i (V^t b)_i / s_i^2.
struct WaveSVD {
    double B[6];  // this lane's row of B V
    double V[6];  // row `lane` of V (lanes 0..5; zero elsewhere)
    double s[6];  // singular values (wave-uniform)
    double tol;   // eps max(6, K) s_max
    int rank;
};

__device__ __forceinline__ void wave_svd(WaveSVD& sv, int lane, int keff) {
#pragma unroll
    for (int i = 0; i < 6; ++i) sv.V[i] = lane == i ? 1.0 : 0.0;
    double fro = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) fro += sv.B[i] * sv.B[i];
    const double small = ALG_EPS * ALG_EPS * uniform(wave_sum(fro));
    for (int sweep = 0; sweep < 40; ++sweep) {
        int rot = 0;
#pragma unroll
        for (int p = 0; p < 5; ++p) {
#pragma unroll
            for (int q = p + 1; q < 6; ++q) {
                double a = sv.B[p] * sv.B[p], b = sv.B[q] * sv.B[q], g = sv.B[p] * sv.B[q];
                wave_sum3(a, b, g);
                a = uniform(a);
                b = uniform(b);
                g = uniform(g);
                if (!(fabs(g) > ALG_EPS * sqrt(a * b)) || fmin(a, b) <= small) continue;
                const double z = (b - a) / (2.0 * g);
                const double t = fabs(z) < 1e150 ? copysign(1.0, z) / (fabs(z) + sqrt(1.0 + z * z)) : 0.5 / z;
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                const double bp = sv.B[p], bq = sv.B[q];
                sv.B[p] = c * bp - sn * bq;
                sv.B[q] = sn * bp + c * bq;
                const double vp = sv.V[p], vq = sv.V[q];
                sv.V[p] = c * vp - sn * vq;
                sv.V[q] = sn * vp + c * vq;
                ++rot;
            }
        }
        if (rot == 0) break;
    }
    double smax = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        sv.s[i] = uniform(sqrt(wave_sum(sv.B[i] * sv.B[i])));
        smax = fmax(smax, sv.s[i]);
    }
    sv.tol = ALG_EPS * static_cast<double>(keff > 6 ? keff : 6) * smax;
    sv.rank = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) sv.rank += sv.s[i] > sv.tol ? 1 : 0;
}

// cond2(G) = (s_max / s_min)^2 of a full-rank system (the rotations leave
// the singular values unordered).
__device__ __forceinline__ double wave_svd_gram_cond(const WaveSVD& sv) {
    double smax = sv.s[0], smin = sv.s[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) {
        smax = fmax(smax, sv.s[i]);
        smin = fmin(smin, sv.s[i]);
    }
    return (smax / smin) * (smax / smin);
}

// (V^t x)_i for a wave-uniform 6-vector x (lane k < 6 holds row k of V).
__device__ __forceinline__ void wave_vt(const WaveSVD& sv, const double x[6], int lane, double out[6]) {
    const double xl = lane == 0 ? x[0] : lane == 1 ? x[1] : lane == 2 ? x[2] : lane == 3 ? x[3]
                    : lane == 4 ? x[4] : lane == 5 ? x[5] : 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) out[i] = uniform(wave_sum(sv.V[i] * xl));
}
// (V x) as a wave-uniform 6-vector.
__device__ __forceinline__ void wave_v(const WaveSVD& sv, const double x[6], double out[6]) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) r += sv.V[i] * x[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k] = lane_value(r, k);
}

// Minimum-norm (least-squares, where rank < 6) solution entry of this lane:
// A_lane = sum over kept i of (B V)_{lane i} (V^t b)_i / s_i^2.
__device__ __forceinline__ double wave_svd_solve(const WaveSVD& sv, const double b[6], int lane) {
    double c[6];
    wave_vt(sv, b, lane, c);
    double A = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        if (sv.s[i] > sv.tol) A += sv.B[i] * (c[i] / (sv.s[i] * sv.s[i]));
    return A;
}

}  // namespace p2m
