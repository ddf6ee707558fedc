// SE(3) on the device, float64.  A twist xi = (rho, phi) holds the
// translational part first; a pose is a row-major 3x4 [R | t] mapping camera
// to world coordinates.  Poses are updated by left multiplication,
// T <- exp(xi^) T (Sec. 5.1 solves for a left increment of the pose).
#pragma once

#include <hip/hip_runtime.h>

namespace gsdf {

__device__ inline void hat3(const double v[3], double K[9]) {
    K[0] = 0.0;   K[1] = -v[2]; K[2] = v[1];
    K[3] = v[2];  K[4] = 0.0;   K[5] = -v[0];
    K[6] = -v[1]; K[7] = v[0];  K[8] = 0.0;
}

__device__ inline void mul33(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// exp(xi^) = [R | V rho] with R = I + A K + B K^2, V = I + B K + C K^2,
// K = phi^, theta = |phi|: A = sin(theta)/theta, B = (1 - cos(theta))/theta^2,
// C = (theta - sin(theta))/theta^3.  Below theta = 0.02 (every Gauss-Newton
// increment of tracking) their Taylor series through theta^8 are exact to
// far below double rounding (the first omitted term is < 1e-24) and avoid
// the sine and cosine.
__device__ inline void se3_exp(const double xi[6], double R[9], double t[3]) {
    const double* rho = xi;
    const double* phi = xi + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 0.02) {
        const double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        A = 1.0 - th2 / 6.0 + t4 / 120.0 - t6 / 5040.0 + t8 / 362880.0;
        B = 0.5 - th2 / 24.0 + t4 / 720.0 - t6 / 40320.0 + t8 / 3628800.0;
        C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t6 / 362880.0 + t8 / 39916800.0;
    } else {
        const double sn = sin(th), cs = cos(th);
        A = sn / th;
        B = (1.0 - cs) / th2;
        C = (th - sn) / (th2 * th);
    }
    double K[9], K2[9], V[9];
    hat3(phi, K);
    mul33(K, K, K2);
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * K[i] + B * K2[i];
        V[i] = I + B * K[i] + C * K2[i];
    }
    for (int i = 0; i < 3; ++i) t[i] = V[3 * i] * rho[0] + V[3 * i + 1] * rho[1] + V[3 * i + 2] * rho[2];
}

// pose <- exp(xi^) pose
__device__ inline void se3_apply_left(const double xi[6], double pose[12]) {
    double R[9], t[3], out[12];
    se3_exp(xi, R, t);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = R[3 * i] * pose[j] + R[3 * i + 1] * pose[4 + j] + R[3 * i + 2] * pose[8 + j];
            if (j == 3) s += t[i];
            out[4 * i + j] = s;
        }
    for (int i = 0; i < 12; ++i) pose[i] = out[i];
}

// Left Jacobian of SE(3), row-major 6x6: [[J, Q], [0, J]] with J the SO(3)
// left Jacobian of phi and Q(rho, phi) the closed form of Barfoot and
// Furgale (IEEE T-RO 2014, "Associating uncertainty with three-dimensional
// poses"):
//   J = I + B K + C K^2,
//   Q = rho^/2 + c1 (K P + P K + K P K) + c2 (K K P + P K K - 3 K P K)
//       + c3 (K P K K + K K P K),
// K = phi^, P = rho^, c1 = (theta - sin)/theta^3,
// c2 = (theta^2 + 2 cos - 2)/(2 theta^4), c3 = (2 theta - 3 sin + theta cos)/(2 theta^5),
// with Taylor series below theta = 0.05, where the closed forms cancel.
// It maps a change of xi to the left increment it causes:
// exp((xi + e)^) ~ exp((Jl e)^) exp(xi^).
__device__ inline void se3_left_jacobian(const double xi[6], double Jl[36]) {
    const double* rho = xi;
    const double* phi = xi + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double B, C, c1, c2, c3;
    if (th < 0.05) {
        const double t4 = th2 * th2;
        B = 0.5 - th2 / 24.0 + t4 / 720.0 - t4 * th2 / 40320.0;
        C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t4 * th2 / 362880.0;
        c1 = C;
        c2 = 1.0 / 24.0 - th2 / 720.0 + t4 / 40320.0 - t4 * th2 / 3628800.0;
        c3 = 1.0 / 120.0 - th2 / 2520.0 + t4 / 120960.0 - t4 * th2 / 9979200.0;
    } else {
        const double sn = sin(th), cs = cos(th);
        const double t3 = th2 * th;
        B = (1.0 - cs) / th2;
        C = (th - sn) / t3;
        c1 = C;
        c2 = (th2 + 2.0 * cs - 2.0) / (2.0 * th2 * th2);
        c3 = (2.0 * th - 3.0 * sn + th * cs) / (2.0 * th2 * t3);
    }
    double K[9], P[9], KK[9], KP[9], PK[9], KPK[9], KKP[9], PKK[9], KPKK[9], KKPK[9];
    hat3(phi, K);
    hat3(rho, P);
    mul33(K, K, KK);
    mul33(K, P, KP);
    mul33(P, K, PK);
    mul33(KP, K, KPK);
    mul33(KK, P, KKP);
    mul33(PK, K, PKK);
    mul33(KPK, K, KPKK);
    mul33(K, KPK, KKPK);
    for (int i = 0; i < 36; ++i) Jl[i] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int e = 3 * i + j;
            const double I = (i == j) ? 1.0 : 0.0;
            const double J = I + B * K[e] + C * KK[e];
            const double Q = 0.5 * P[e] + c1 * (KP[e] + PK[e] + KPK[e]) +
                             c2 * (KKP[e] + PKK[e] - 3.0 * KPK[e]) + c3 * (KPKK[e] + KKPK[e]);
            Jl[6 * i + j] = J;
            Jl[6 * (i + 3) + (j + 3)] = J;
            Jl[6 * i + (j + 3)] = Q;
        }
}

}  // namespace gsdf
