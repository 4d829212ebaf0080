// Velocity-Verlet integrator kernels.  The paper runs its MD inside an
// external engine and states no integrator; the MD step here is plain NVE
// velocity Verlet with an optional affine engineering strain (the constant
// strain-rate loading of Sec. III.C.5).
#include "nep_internal.h"

namespace nep {




__global__ __launch_bounds__(BLOCK) void k_kick_drift(KickDriftArgs a) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    // every read is issued before the freeze test (nothing is written before
    // it), so that the test's latency overlaps theirs
    const bool frozen = (a.status[0] & FREEZE_MASK) != 0;
    int t = 0;
    BeadIn in{};
    if (i < a.n) {
        t = min((int)a.type[i], a.T - 1);
        in = kick_drift_read(i, a.n, a.x, a.y, a.z, a.v, a.F, a.ref);
    }
    // first level of the previous step's reduction: this workgroup's range of
    // the gather's block partials, summed in order
    double acc = 0.0;
    const bool sums = a.prev_partial && threadIdx.x < NPART_NVE;
    if (sums) {
        const int per = (a.prev_blocks + gridDim.x - 1) / gridDim.x;
        const int b0 = blockIdx.x * per, b1 = min(b0 + per, a.prev_blocks);
        for (int b = b0; b < b1; ++b) acc += a.prev_partial[(size_t)b * NPART + threadIdx.x];
    }
    if (frozen) return;  // lists invalid: leave the state untouched (uniform)
    // the pair test's other counter starts the next step from zero, and the
    // verdict of the last step's test is spent
    if (a.fast && i == 0) {
        a.fast[a.parity ^ 1] = 0;
        a.fast[3] = 0;
    }
    if (sums) a.pre[(size_t)blockIdx.x * NPART + threadIdx.x] = acc;
    // the cell counts of a build later in this step start from zero (cleared
    // here rather than by a launch of its own, which every step would pay)
    if (a.cell_count)
        for (int c = i; c < a.ncell; c += gridDim.x * BLOCK) a.cell_count[c] = 0;
    float d2 = 0.0f;
    if (i < a.n) {
        const float k = a.half_dt_accel * a.inv_mass[t];
        d2 = kick_drift_write(in, i, a.n, t, k, a.dt, a.lam[0], a.lam[1], a.lam[2], a.vh, a.pos4, a.ref);
        // a bead past tau joins the pair test's list (past FAST_CAP only counted)
        if (a.fast && d2 >= a.tau2) {
            const int q = atomicAdd(&a.fast[a.parity], 1);
            if (q < FAST_CAP) a.fast[4 + q] = i;
        }
    }
    const float2 tt = block_top2(d2, 0.0f);
    if (threadIdx.x == 0) a.top2[blockIdx.x] = tt;
}

// one workgroup: the merge kernel (gate_body)
__global__ __launch_bounds__(BLOCK) void k_gate(KickDriftArgs a, int nblocks) { gate_body(a, nblocks); }

hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t s, bool gate) {
    if (a.n == 0) return hipSuccess;
    const int nb = (a.n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_kick_drift, dim3(nb), dim3(BLOCK), 0, s, a);
    if (gate) hipLaunchKernelGGL(k_gate, dim3(1), dim3(BLOCK), 0, s, a, nb);
    return hipGetLastError();
}


// Gathers every per-bead array into the order given by src through the
// staging area, then writes it back in place.

__global__ void k_permute_gather(PermuteArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n) return;
    const int n = a.n;
    const int i = a.src[s];
    float *t = a.tmp;
    t[s] = a.x[i];
    t[n + s] = a.y[i];
    t[2 * n + s] = a.z[i];
    for (int d = 0; d < 3; ++d) {
        if (a.v) t[(3 + d) * (size_t)n + s] = a.v[(size_t)d * n + i];
        if (a.F) t[(6 + d) * (size_t)n + s] = a.F[(size_t)d * n + i];
    }
    if (a.U) t[9 * (size_t)n + s] = a.U[i];
    if (a.perm) reinterpret_cast<int32_t *>(t)[10 * (size_t)n + s] = a.perm[i];
    reinterpret_cast<uint8_t *>(t + 11 * (size_t)n)[s] = a.type[i];
}

__global__ void k_permute_scatter(PermuteArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n) return;
    const int n = a.n;
    const float *t = a.tmp;
    a.x[s] = t[s];
    a.y[s] = t[n + s];
    a.z[s] = t[2 * n + s];
    for (int d = 0; d < 3; ++d) {
        if (a.v) a.v[(size_t)d * n + s] = t[(3 + d) * (size_t)n + s];
        if (a.F) a.F[(size_t)d * n + s] = t[(6 + d) * (size_t)n + s];
    }
    if (a.U) a.U[s] = t[9 * (size_t)n + s];
    if (a.perm) a.perm[s] = reinterpret_cast<const int32_t *>(t)[10 * (size_t)n + s];
    a.type[s] = reinterpret_cast<const uint8_t *>(t + 11 * (size_t)n)[s];
}

hipError_t launch_permute(const PermuteArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 g((a.n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_permute_gather, g, dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_permute_scatter, g, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace nep
