// pot_register.hip -- rigid point-cloud registration through POT: the outer
// loop of Section 4 ("Point Cloud Registration") and its appendix.  Each
// registration moves the cloud Y by the current map F(y) = R y + t (a
// kernel), solves POT between X and F(Y) (pot_solve's path, points cost,
// warm-started from the previous registration's duals rescaled to the new
// entropic parameter), takes the rounded plan's moments on the device, and
// updates the map on the host by the weighted-barycentre alignment: the
// rotation that maximises tr(R^T H) for the centred cross-covariance H,
// found as the leading eigenvector of Horn's 4 x 4 quaternion matrix (a
// published closed form of the same optimum as the appendix's SVD).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "pot_internal.h"

namespace pot {

// y_k = R y + t (FP64 arithmetic, stored in FP32: the precision of the clouds)
__global__ void transform_points(const float* y, float* yk, int m, RigidMap F) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const double a = y[3 * j], b = y[3 * j + 1], c = y[3 * j + 2];
    for (int r = 0; r < 3; ++r)
        yk[3 * j + r] = (float)(fma(F.R[3 * r], a, fma(F.R[3 * r + 1], b, fma(F.R[3 * r + 2], c, F.t[r]))));
}

// warm start of the next registration: the potentials in cost units kept,
// the log-scalings rescaled by gamma_prev / gamma_new
__global__ void scale_duals(const double* u, const double* v, double* u0, double* v0, int n, int m, double sc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) u0[k] = u[k] * sc;
    if (k < m) v0[k] = v[k] * sc;
}

// history of a registration: the moved cloud and the solve's duals
__global__ void record_step(const float* yk, const double* u, const double* v, int n, int m, double w,
                            float* yh, double* dh) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (yh && k < 3 * m) yh[k] = yk[k];
    if (dh) {
        if (k < n) dh[k] = u[k];
        if (k < m) dh[n + k] = v[k];
        if (k == 0) dh[n + m] = w;
    }
}

hipError_t launch_transform(const float* y, float* yk, int m, const RigidMap& F, hipStream_t st) {
    transform_points<<<(m + 255) / 256, 256, 0, st>>>(y, yk, m, F);
    return hipGetLastError();
}

hipError_t launch_scale_duals(const double* u, const double* v, double* u0, double* v0, int n, int m, double sc,
                              hipStream_t st) {
    const int len = std::max(n, m);
    scale_duals<<<(len + 255) / 256, 256, 0, st>>>(u, v, u0, v0, n, m, sc);
    return hipGetLastError();
}

hipError_t launch_record_step(const float* yk, const double* u, const double* v, int n, int m, double w, float* yh,
                              double* dh, hipStream_t st) {
    const int len = std::max(3 * m, std::max(n, m));
    record_step<<<(len + 255) / 256, 256, 0, st>>>(yk, u, v, n, m, w, yh, dh);
    return hipGetLastError();
}

// Leading eigenvector of a symmetric 4 x 4 matrix by cyclic Jacobi rotations.
static void jacobi4_leading(double A[4][4], double q[4]) {
    double V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 4; ++p)
            for (int r = p + 1; r < 4; ++r) off += A[p][r] * A[p][r];
        if (off == 0.0) break;
        for (int p = 0; p < 4; ++p)
            for (int r = p + 1; r < 4; ++r) {
                if (A[p][r] == 0.0) continue;
                // rotation that zeroes A[p][r] (Golub & Van Loan, symmetric Schur decomposition)
                const double tau = (A[r][r] - A[p][p]) / (2.0 * A[p][r]);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < 4; ++k) {
                    const double akp = A[k][p], akr = A[k][r];
                    A[k][p] = c * akp - s * akr;
                    A[k][r] = s * akp + c * akr;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = A[p][k], ark = A[r][k];
                    A[p][k] = c * apk - s * ark;
                    A[r][k] = s * apk + c * ark;
                }
                for (int k = 0; k < 4; ++k) {
                    const double vkp = V[k][p], vkr = V[k][r];
                    V[k][p] = c * vkp - s * vkr;
                    V[k][r] = s * vkp + c * vkr;
                }
            }
    }
    int best = 0;
    for (int k = 1; k < 4; ++k)
        if (A[k][k] > A[best][best]) best = k;
    for (int k = 0; k < 4; ++k) q[k] = V[k][best];
}

// The rotation R in SO(3) maximising tr(R^T H) (H row-major): with
// S = H^T (S_ab = sum w y_a x_b for the map y -> x), the unit quaternion of
// R is the leading eigenvector of Horn's symmetric matrix N(S).
void rigid_align(const double* H, double* R) {
    double S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = H[3 * b + a];
    const double sxx = S[0][0], sxy = S[0][1], sxz = S[0][2];
    const double syx = S[1][0], syy = S[1][1], syz = S[1][2];
    const double szx = S[2][0], szy = S[2][1], szz = S[2][2];
    double N[4][4] = {
        {sxx + syy + szz, syz - szy, szx - sxz, sxy - syx},
        {syz - szy, sxx - syy - szz, sxy + syx, szx + sxz},
        {szx - sxz, sxy + syx, -sxx + syy - szz, syz + szy},
        {sxy - syx, szx + sxz, syz + szy, -sxx - syy + szz}};
    double q[4];
    jacobi4_leading(N, q);
    const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
    R[0] = w * w + x * x - y * y - z * z;
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (y * x + w * z);
    R[4] = w * w - x * x + y * y - z * z;
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (z * x - w * y);
    R[7] = 2.0 * (z * y + w * x);
    R[8] = w * w - x * x - y * y + z * z;
}

}  // namespace pot
