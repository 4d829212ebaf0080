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
    int t = min((int)a.type[i], a.T - 1);
    const float k = a.half_dt_accel * a.inv_mass[t];
    // every lane that sees a bead too far writes the same value
    if (kick_drift_bead(i, a.n, t, k, a.dt, a.lam[0], a.lam[1], a.lam[2], a.x, a.y, a.z, a.v, a.vh, a.F,
                        a.pos4, a.ref, a.gate2))
        a.ctrl[0] = 1;
}

hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_drift, dim3((a.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace nep
