// Velocity-Verlet integrator kernels.  The paper runs its MD inside an
// external engine and states no integrator; the MD step here is plain NVE
// velocity Verlet with an optional affine engineering strain (the constant
// strain-rate loading of Sec. III.C.5).
#include "nep_internal.h"

namespace nep {




__global__ void k_kick_drift(KickDriftArgs a) {
    if (a.status[0] & FREEZE_MASK) return;  // lists invalid: leave the state untouched
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int n = a.n;
    int t = min((int)a.type[i], a.T - 1);
    float k = a.half_dt_accel * a.inv_mass[t];
    float vx = a.v[i] + k * a.F[i];
    float vy = a.v[n + i] + k * a.F[n + i];
    float vz = a.v[2 * n + i] + k * a.F[2 * n + i];
    a.vh[i] = vx;
    a.vh[n + i] = vy;
    a.vh[2 * n + i] = vz;
    float x = (a.x[i] + a.dt * vx) * a.lam[0];
    float y = (a.y[i] + a.dt * vy) * a.lam[1];
    float z = (a.z[i] + a.dt * vz) * a.lam[2];
    float rx = a.ref[i] * a.lam[0], ry = a.ref[n + i] * a.lam[1], rz = a.ref[2 * n + i] * a.lam[2];
    a.ref[i] = rx;
    a.ref[n + i] = ry;
    a.ref[2 * n + i] = rz;
    float ddx = x - rx, ddy = y - ry, ddz = z - rz;
    // every lane that sees a bead too far writes the same value
    if (ddx * ddx + ddy * ddy + ddz * ddz > a.gate2) a.ctrl[0] = 1;
    a.pos4[i] = make_float4(x, y, z, (float)t);
}

hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_drift, dim3((a.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace nep
