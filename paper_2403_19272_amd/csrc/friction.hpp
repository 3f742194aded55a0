// Lagged friction of an obstacle contact (device side; included by the
// kernels that sum collision weights, so that all of them sum the same bits).
//
// Section 8.4 of the paper drapes a cloth with a lagged friction Hessian at
// every local/global iteration.  Here a contact with a spinning or fixed
// analytic obstacle in the contact band gets, besides its barrier weight w
// and projection, a friction weight
//   wf = mu lambda f1(|u_T|) / |u_T|,   lambda = w (R + d_hat - |radial|),
// with the tangential slip u_T of (x - x*) - h v_s over the step (x* the
// step's start, v_s = omega R (axis x n) the surface velocity, n the unit
// radial direction) and the smoothed Coulomb factor
//   f1(y) / y = 2 / eps - y / eps^2 (y < eps),  1 / y (y >= eps),
// and the target x - u_T: the force wf |u_T| is mu lambda while slipping
// and proportional to the slip while sticking.  All of it is evaluated from
// the current iterate (lagged), in FP64.
#pragma once

#include "scene.hpp"

namespace cloth {

// The radial vector of x from an obstacle (the axis part removed for a
// cylinder) and its length, with the written operation order (no
// contraction), so that every kernel that needs it gets the same bits.
__device__ __forceinline__ double obstacle_radial(const ObstD& o, float x0, float x1, float x2, double& ox,
                                                  double& oy, double& oz) {
#pragma clang fp contract(off)
    ox = x0 - o.c[0];
    oy = x1 - o.c[1];
    oz = x2 - o.c[2];
    if (o.kind == CLOTH_CYLINDER) {
        const double ax = ox * o.a[0] + oy * o.a[1] + oz * o.a[2];
        ox -= ax * o.a[0];
        oy -= ax * o.a[1];
        oz -= ax * o.a[2];
    }
    return sqrt(ox * ox + oy * oy + oz * oz);
}

// (ox, oy, oz): the radial vector of x from the obstacle (axis part removed
// for a cylinder), rad its length, w the barrier weight, (x0, x1, x2) the
// iterate and (s0, s1, s2) the step's start.  Returns wf and the slip.
__device__ __forceinline__ double obstacle_friction(const Dev& d, const ObstD& o, float w, double ox, double oy,
                                                    double oz, double rad, double x0, double x1, double x2,
                                                    double s0, double s1, double s2, double& ux, double& uy,
                                                    double& uz) {
#pragma clang fp contract(off)
    ux = uy = uz = 0.0;
    if (d.mu <= 0.0f || !(rad > 0) || !(rad - o.R < d.dhat)) return 0.0;
    const double inv = 1.0 / rad;
    const double nx = ox * inv, ny = oy * inv, nz = oz * inv;
    // h v_s = (omega h) R (a x n)
    const double k = o.wh * o.R;
    const double vx = k * (o.a[1] * nz - o.a[2] * ny);
    const double vy = k * (o.a[2] * nx - o.a[0] * nz);
    const double vz = k * (o.a[0] * ny - o.a[1] * nx);
    double px = (x0 - s0) - vx, py = (x1 - s1) - vy, pz = (x2 - s2) - vz;
    const double pn = px * nx + py * ny + pz * nz;
    px -= pn * nx;
    py -= pn * ny;
    pz -= pn * nz;
    const double y = sqrt(px * px + py * py + pz * pz);
    const double lam = (double)w * (o.R + d.dhat - rad);
    const double eps = d.feps;
    const double f = y < eps ? (2.0 / eps - y / (eps * eps)) : 1.0 / y;
    ux = px;
    uy = py;
    uz = pz;
    return (double)d.mu * lam * f;
}

}  // namespace cloth
