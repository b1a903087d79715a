// Boundary assembly of the wall model (Algorithm 1, "Boundary assembly";
// Section 3.2 names a law-of-the-wall model).  One thread per wall face:
//   exchange point: vertex average of the face's volume element, where the
//     linear interpolant of the velocity is the mean of its nodal values;
//   wall distance y: from that point to the plane of the face (unit normal
//     n from the face's edge or diagonal cross product);
//   tangential velocity u_t = u_e - (u_e . n) n, U = |u_t|;
//   friction velocity from Reichardt's law U / u_tau = f(y u_tau / nu)
//     (kappa 0.41, C1 7.8, chi 11) by Newton's method from the viscous-
//     sublayer value sqrt(nu U / y);
//   traction t = -u_tau^2 u_t / U, added to the face nodes with the face
//     integrals of their shape functions (triangle: A/3; bilinear quad: 2 x 2
//     Gauss).  Faces sharing a node add with FP64 atomics.
#include "common.hpp"

namespace lesasm {

namespace {

constexpr double kKappa = 0.41, kC1 = 7.8, kChi = 11.0;

__device__ __forceinline__ double wall_law(double yp) {
    return log(1.0 + kKappa * yp) / kKappa + kC1 * (1.0 - exp(-yp / kChi) - (yp / kChi) * exp(-yp / 3.0));
}

__device__ __forceinline__ double wall_law_slope(double yp) {
    return 1.0 / (1.0 + kKappa * yp) +
           kC1 * (exp(-yp / kChi) / kChi - exp(-yp / 3.0) / kChi + (yp / kChi) * exp(-yp / 3.0) / 3.0);
}

__device__ double friction_velocity(double U, double y, double nu) {
    if (!(U > 0.0)) return 0.0;
    double ut = sqrt(nu * U / y);
    for (int it = 0; it < 100; ++it) {
        const double yp = y * ut / nu;
        const double f = wall_law(yp);
        const double step = (ut * f - U) / (f + yp * wall_law_slope(yp));
        ut -= step;
        if (fabs(step) <= 1e-15 * ut) break;
    }
    return ut;
}

__device__ __forceinline__ void cross(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ __launch_bounds__(256) void k_wall(const int32_t *__restrict__ fg, const int32_t *__restrict__ ff,
                                              const int32_t *__restrict__ eg, const int32_t *__restrict__ ef,
                                              const double *__restrict__ xyz, const double *__restrict__ u, double nu,
                                              double *__restrict__ rhs, int n) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    // exchange point and velocity
    double xe[3] = {0, 0, 0}, ue[3] = {0, 0, 0};
    int ne = 0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int g = eg[8 * f + a];
        if (g < 0) continue;
        const int q = ef[8 * f + a];
        ++ne;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xe[k] += xyz[3 * (size_t)g + k];
            ue[k] += u[3 * (size_t)q + k];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        xe[k] /= ne;
        ue[k] /= ne;
    }
    // face geometry
    const int nf = fg[4 * f + 3] < 0 ? 3 : 4;
    double xf[4][3], xc[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (b == 3 && nf == 3) break;
        const int g = fg[4 * f + b];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xf[b][k] = xyz[3 * (size_t)g + k];
            xc[k] += xf[b][k] / nf;
        }
    }
    double c[3], wa[4];
    if (nf == 3) {
        double d1[3], d2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            d1[k] = xf[1][k] - xf[0][k];
            d2[k] = xf[2][k] - xf[0][k];
        }
        cross(d1, d2, c);
        const double area = 0.5 * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        wa[0] = wa[1] = wa[2] = area / 3.0;
        wa[3] = 0.0;
    } else {
        double d1[3], d2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            d1[k] = xf[2][k] - xf[0][k];
            d2[k] = xf[3][k] - xf[1][k];
        }
        cross(d1, d2, c);
        const double s[4] = {-1, 1, 1, -1}, t[4] = {-1, -1, 1, 1};
        const double gq = 0.577350269189625764509148780502;
        wa[0] = wa[1] = wa[2] = wa[3] = 0.0;
#pragma unroll
        for (int gi = 0; gi < 2; ++gi)
#pragma unroll
            for (int gj = 0; gj < 2; ++gj) {
                const double xi = gi ? gq : -gq, eta = gj ? gq : -gq;
                double dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        dx[k] += 0.25 * s[a] * (1.0 + t[a] * eta) * xf[a][k];
                        dy[k] += 0.25 * t[a] * (1.0 + s[a] * xi) * xf[a][k];
                    }
                double cc[3];
                cross(dx, dy, cc);
                const double jac = sqrt(cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2]);
#pragma unroll
                for (int a = 0; a < 4; ++a) wa[a] += 0.25 * (1.0 + s[a] * xi) * (1.0 + t[a] * eta) * jac;
            }
    }
    const double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double nrm[3], y = 0.0, un = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        nrm[k] = c[k] / len;
        y += nrm[k] * (xe[k] - xc[k]);
        un += nrm[k] * ue[k];
    }
    y = fabs(y);
    double ut[3], U = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ut[k] = ue[k] - un * nrm[k];
        U += ut[k] * ut[k];
    }
    U = sqrt(U);
    if (!(U > 0.0)) return;
    const double utau = friction_velocity(U, y, nu);
    const double sc = -utau * utau / U;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (b == 3 && nf == 3) break;
        const size_t q = (size_t)ff[4 * f + b];
#pragma unroll
        for (int k = 0; k < 3; ++k) unsafeAtomicAdd(rhs + 3 * q + k, sc * ut[k] * wa[b]);
    }
}

}  // namespace

int launch_wall(lesasm_mesh *m, const double *u, double nu, double *rhs, hipStream_t s) {
    const int n = (int)m->n_wall;
    hipLaunchKernelGGL(k_wall, dim3((n + 255) / 256), dim3(256), 0, s, m->d_wall_fg, m->d_wall_ff, m->d_wall_eg,
                       m->d_wall_ef, m->d_xyz, u, nu, rhs, n);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

}  // namespace lesasm
