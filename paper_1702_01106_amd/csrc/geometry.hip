// Metric tables for modified Kerr-Schild coordinates (a1, Sec. 2.1):
// r = exp(X1), theta = pi X2 + (1-h)/2 sin(2 pi X2), phi = X3, with
// L = diag(1, r, dtheta/dX2, 1).
//
// The metric depends on (X1, X2) only, so the tables are two-dimensional:
// one entry per (i, j) of the ghosted grid, shared by every k.  Entries:
// the seven nonzero g_{mu nu}, the seven nonzero g^{mu nu} (closed-form
// inverse of Kerr-Schild), sqrt(-g) and the lapse, at zone centres and at the
// low faces in X1, X2 and X3; and Gamma^l_{m n} at zone centres from
// fourth-order central differences of g_{mu nu}.
//
// Near the axis sin^2(theta) is kept >= 1e-24 so the inverse stays finite;
// theta itself is not clamped, so ghost zones across the axis see the mirror
// image of the metric (sin^2 and cos are even about theta = 0 and pi).
#include <hip/hip_runtime.h>

#include "grim_internal.h"

namespace grim {

namespace {

struct MKS {
    double a, h;
};

// g_{mu nu} in MKS at (X1, X2), full 4x4.
__device__ void mks_gcov(const MKS& p, double X1, double X2, double g[4][4])
{
    const double r = exp(X1);
    const double th = M_PI * X2 + 0.5 * (1.0 - p.h) * sin(2.0 * M_PI * X2);
    const double dth = M_PI * (1.0 + (1.0 - p.h) * cos(2.0 * M_PI * X2));
    const double ct = cos(th);
    const double s2 = fmax(sin(th) * sin(th), 1e-24);
    const double a2 = p.a * p.a;
    const double Sig = r * r + a2 * ct * ct;
    const double z = 2.0 * r / Sig;
    const double Ld[4] = {1.0, r, dth, 1.0};
    double k[4][4] = {};
    k[0][0] = -(1.0 - z);
    k[0][1] = k[1][0] = z;
    k[0][3] = k[3][0] = -p.a * z * s2;
    k[1][1] = 1.0 + z;
    k[1][3] = k[3][1] = -p.a * s2 * (1.0 + z);
    k[2][2] = Sig;
    k[3][3] = s2 * (Sig + a2 * s2 * (1.0 + z));
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) g[m][n] = k[m][n] * Ld[m] * Ld[n];
}

// Closed-form g^{mu nu} of Kerr-Schild mapped to MKS, sqrt(-g) and the lapse.
__device__ void mks_gcon(const MKS& p, double X1, double X2, double u[4][4], double& gdet, double& alpha)
{
    const double r = exp(X1);
    const double th = M_PI * X2 + 0.5 * (1.0 - p.h) * sin(2.0 * M_PI * X2);
    const double dth = M_PI * (1.0 + (1.0 - p.h) * cos(2.0 * M_PI * X2));
    const double ct = cos(th);
    const double s2 = fmax(sin(th) * sin(th), 1e-24);
    const double a2 = p.a * p.a;
    const double Sig = r * r + a2 * ct * ct;
    const double Del = r * r - 2.0 * r + a2;
    const double Ld[4] = {1.0, r, dth, 1.0};
    double k[4][4] = {};
    k[0][0] = -(1.0 + 2.0 * r / Sig);
    k[0][1] = k[1][0] = 2.0 * r / Sig;
    k[1][1] = Del / Sig;
    k[1][3] = k[3][1] = p.a / Sig;
    k[2][2] = 1.0 / Sig;
    k[3][3] = 1.0 / (Sig * s2);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) u[m][n] = k[m][n] / (Ld[m] * Ld[n]);
    gdet = Sig * sqrt(s2) * r * fabs(dth);
    alpha = 1.0 / sqrt(1.0 + 2.0 * r / Sig);
}

__device__ void store_point(const MKS& p, double X1, double X2, double* t, size_t idx, size_t stride)
{
    double g[4][4], u[4][4], gd, al;
    mks_gcov(p, X1, X2, g);
    mks_gcon(p, X1, X2, u, gd, al);
    const int pairs[7][2] = {{0, 0}, {0, 1}, {0, 3}, {1, 1}, {1, 3}, {2, 2}, {3, 3}};
    for (int q = 0; q < 7; ++q) {
        t[q * stride + idx] = g[pairs[q][0]][pairs[q][1]];
        t[(7 + q) * stride + idx] = u[pairs[q][0]][pairs[q][1]];
    }
    t[14 * stride + idx] = gd;
    t[15 * stride + idx] = al;
}

__global__ void k_geometry(Layout L, MKS p, double* centre, double* f1, double* f2, double* f3, double* conn)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long npt = (long)L.N[0] * L.N[1];
    if (t >= npt) return;
    const int i = (int)(t % L.N[0]);
    const int j = (int)(t / L.N[0]);
    const double X1 = L.xs[0] + (i - L.g[0] + 0.5) * L.dx[0];
    const double X2 = L.xs[1] + (j - L.g[1] + 0.5) * L.dx[1];
    const size_t s = (size_t)npt;
    store_point(p, X1, X2, centre, (size_t)t, s);
    store_point(p, X1 - 0.5 * L.dx[0], X2, f1, (size_t)t, s);
    store_point(p, X1, X2 - 0.5 * L.dx[1], f2, (size_t)t, s);
    store_point(p, X1, X2, f3, (size_t)t, s);

    // d_k g_{mn}: zero for k = 0, 3 (stationary, axisymmetric); fourth-order
    // central differences in X1 and X2.
    double dg[4][4][4] = {};
    const double hd = 1e-3;
    for (int k = 1; k <= 2; ++k) {
        double gp2[4][4], gp1[4][4], gm1[4][4], gm2[4][4];
        const double e1 = k == 1 ? hd : 0.0, e2 = k == 2 ? hd : 0.0;
        mks_gcov(p, X1 + 2 * e1, X2 + 2 * e2, gp2);
        mks_gcov(p, X1 + e1, X2 + e2, gp1);
        mks_gcov(p, X1 - e1, X2 - e2, gm1);
        mks_gcov(p, X1 - 2 * e1, X2 - 2 * e2, gm2);
        for (int m = 0; m < 4; ++m)
            for (int n = 0; n < 4; ++n)
                dg[k][m][n] = (8.0 * (gp1[m][n] - gm1[m][n]) - (gp2[m][n] - gm2[m][n])) / (12.0 * hd);
    }
    double u[4][4], gd, al;
    mks_gcon(p, X1, X2, u, gd, al);
    // Gamma^l_{m n} = Gamma^l_{n m}: computed for m <= n and stored at both,
    // so the table is symmetric to the bit
    for (int l = 0; l < 4; ++l)
        for (int m = 0; m < 4; ++m)
            for (int n = m; n < 4; ++n) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += u[l][k] * (dg[m][k][n] + dg[n][k][m] - dg[k][m][n]);
                conn[(size_t)(l * 16 + m * 4 + n) * s + t] = 0.5 * acc;
                conn[(size_t)(l * 16 + n * 4 + m) * s + t] = 0.5 * acc;
            }
}

}  // namespace

hipError_t build_geometry(const Layout& L, double spin, double h, double* centre, double* face[3], double* conn,
                          hipStream_t st)
{
    const long npt = (long)L.N[0] * L.N[1];
    MKS p{spin, h};
    hipLaunchKernelGGL(k_geometry, dim3((unsigned)((npt + 127) / 128)), dim3(128), 0, st, L, p, centre, face[0],
                       face[1], face[2], conn);
    return hipGetLastError();
}

}  // namespace grim
