// Ensemble steps of the MD integrator: the NVT/NPT runs the paper equilibrates
// with (Sec. III.A.1, III.C.3) and the HNEMD heat-current runs (Sec. III.B.3),
// which it performs in an external engine without naming the algorithms.
// Taken here: Berendsen or Bussi (stochastic velocity rescaling) thermostats
// applied after the second half-kick, and the HNEMD driving force of Fan et
// al. (Phys. Rev. B 99, 064308), F_i^ext = W_i^T F_e minus its mean over the
// beads, with the potential heat current J = sum_i W_i v_i.  The per-call
// Berendsen barostat needs no kernel of its own: the host applies its scale
// factor like an affine strain, and the pressure comes from the sums below.
//
// After the ensemble-mode gather (forces, virial, drive; no kick):
//   k_ens_reduce   one workgroup: energy, virial and pair-count sums, the MD
//                  bookkeeping, the mean drive
//   k_con_project  one thread per bead (constrained label runs, Sec. II.C.1):
//                  the bead's total atomic force and virial accumulated
//                  (Eqs. 12, 14) and the centre-of-mass constraint force
//   k_ens_finish   one thread per bead: drive without its mean, second
//                  half-kick, commit of x and v, per-block kinetic tensor and
//                  heat current
//   k_ens_thermo   one workgroup: thermostat factor, traces, pressure sum
//   k_ens_scale    one thread per bead: v *= lambda (thermostat runs only)
#include "nep_internal.h"

namespace nep {

constexpr int ENS_P2 = 8;  // finish-block record: K, Kxx, Kyy, Kzz, Jx, Jy, Jz, pad

__global__ __launch_bounds__(BLOCK) void k_ens_reduce(EnsArgs e) {
    reduce_partials<NPART>(e.partial, e.nblocks, nullptr, nullptr, nullptr, e.E_slot, nullptr, e.W_slot, e.counts,
                           e.status, e.ctrl, e.next_gate, e.ens, 1.0 / (double)e.n);
}

// one thread per bead (a contiguous range of atoms): the bead's total atomic
// force and virial, added to the accumulators when acc is set, and the
// constraint force -(m_i/M_I) F_I on each of its atoms, which leaves the
// bead's centre of mass unaccelerated
__global__ __launch_bounds__(BLOCK) void k_con_project(EnsArgs e, int acc) {
    if (e.status[0] & FREEZE_MASK) return;
    const int g = blockIdx.x * BLOCK + threadIdx.x;
    if (g >= e.n_groups) return;
    const int n = e.n;
    // a range outside [0, n) is clamped (the caller's table is not trusted)
    const int a0 = max(0, min(e.group_start[g], n)), a1 = max(a0, min(e.group_start[g + 1], n));
    double FI[3] = {0.0, 0.0, 0.0}, MI = 0.0;
    for (int i = a0; i < a1; ++i) {
        MI += (double)e.mass[min((int)e.type[i], e.T - 1)];
        for (int b = 0; b < 3; ++b) FI[b] += (double)e.F[(size_t)b * n + i];
    }
    if (acc) {
        for (int b = 0; b < 3; ++b) e.F_sum[(size_t)b * e.n_groups + g] += FI[b];
        for (int c = 0; c < 9; ++c) {
            double w = 0.0;
            for (int i = a0; i < a1; ++i) w += (double)e.Wb[(size_t)c * n + i];
            e.W_sum[(size_t)c * e.n_groups + g] += w;
        }
    }
    if (!(MI > 0.0)) return;
    for (int i = a0; i < a1; ++i) {
        const double w = (double)e.mass[min((int)e.type[i], e.T - 1)] / MI;
        for (int b = 0; b < 3; ++b) {
            float *f = e.F + (size_t)b * n + i;
            *f = (float)((double)*f - w * FI[b]);
        }
    }
}

hipError_t launch_constraint_project(const EnsArgs &e, hipStream_t s) {
    if (e.n == 0 || e.n_groups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_con_project, dim3((e.n_groups + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, e, 0);
    return hipGetLastError();
}

__global__ __launch_bounds__(BLOCK) void k_ens_finish(EnsArgs e) {
    __shared__ double red[ENS_P2][BLOCK / 64];
    if (e.status[0] & FREEZE_MASK) return;  // uniform over the grid
    const int n = e.n;
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    double acc[ENS_P2] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        float f[3] = {e.F[i], e.F[n + i], e.F[2 * n + i]};
        if (e.hn) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                f[b] = (float)((double)f[b] - e.ens[b]);
                e.F[(size_t)b * n + i] = f[b];
            }
        }
        const int t = min((int)e.type[i], e.T - 1);
        const float k = e.half_dt_accel * e.inv_mass[t];
        float v[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            v[b] = e.vh[(size_t)b * n + i] + k * f[b];
            e.v[(size_t)b * n + i] = v[b];
        }
        const float4 p = e.pos4[i];
        e.x[i] = p.x;
        e.y[i] = p.y;
        e.z[i] = p.z;
        const double hm = 0.5 * (double)e.mass[t] / (double)ACCEL;
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[1 + b] = hm * (double)v[b] * (double)v[b];
        acc[0] = acc[1] + acc[2] + acc[3];
        if (e.hn) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float j = 0.0f;
#pragma unroll
                for (int b = 0; b < 3; ++b) j += e.Wb[(size_t)(3 * a + b) * n + i] * v[b];
                acc[4 + a] = (double)j;
            }
        }
    }
    // fixed-order block sums: butterfly in each wave, then the waves in order
#pragma unroll
    for (int c = 0; c < ENS_P2; ++c) {
        double s = acc[c];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
        if (__lane_id() == 0) red[c][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x < ENS_P2) {
        double s = red[threadIdx.x][0];
#pragma unroll
        for (int w = 1; w < BLOCK / 64; ++w) s += red[threadIdx.x][w];
        e.partial2[(size_t)blockIdx.x * ENS_P2 + threadIdx.x] = s;
    }
}

// Thermostat factor from the kinetic energy K of the step (N_f = 3n - 3):
// Berendsen lambda^2 = 1 + (dt/tau)(T0/T - 1); Bussi: the exact update of the
// kinetic energy over dt, K' = c K + (1-c) Kbar (S + R^2)/N_f
// + 2 R sqrt(c (1-c) K Kbar / N_f), c = exp(-dt/tau), Kbar = N_f k_B T0 / 2,
// lambda = sqrt(K'/K) with the sign of R + sqrt(c N_f K / ((1-c) Kbar)).
__device__ __forceinline__ double thermostat_factor(const EnsArgs &e, double K) {
    if (!e.thermostat || e.n < 2 || !(K > 0.0)) return 1.0;
    const double Nf = 3.0 * e.n - 3.0;
    if (e.thermostat == 1) {
        const double T = 2.0 * K / (Nf * e.kB);
        const double l2 = 1.0 + e.dt / e.tau_T * (e.T_target / T - 1.0);
        return sqrt(l2 > 0.0 ? l2 : 0.0);
    }
    const double Kbar = 0.5 * Nf * e.kB * e.T_target;
    const double R = e.noise[0], S = e.noise[1];
    const double c = exp(-e.dt / e.tau_T);
    const double Kn = c * K + (1.0 - c) * Kbar * (S + R * R) / Nf + 2.0 * R * sqrt(c * (1.0 - c) * K * Kbar / Nf);
    double lam = sqrt(Kn > 0.0 ? Kn / K : 0.0);
    if (R + sqrt(c * Nf * K / ((1.0 - c) * Kbar)) < 0.0) lam = -lam;
    return lam;
}

__global__ __launch_bounds__(BLOCK) void k_ens_thermo(EnsArgs e) {
    __shared__ double red[ENS_P2][BLOCK];
    if (e.status[0] & FREEZE_MASK) return;
    double acc[ENS_P2] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < e.nb2; b += BLOCK) {
#pragma unroll
        for (int c = 0; c < ENS_P2; ++c) acc[c] += e.partial2[(size_t)b * ENS_P2 + c];
    }
#pragma unroll
    for (int c = 0; c < ENS_P2; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < ENS_P2; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double K = red[0][0];
        const double lam = thermostat_factor(e, K);
        const double l2 = lam * lam;
        e.ens[12] = lam;
        if (e.K_slot) *e.K_slot = l2 * K;
        if (e.J_slot)
            for (int a = 0; a < 3; ++a) e.J_slot[a] = lam * red[4 + a][0];
        // diagonal pressure (2 K_dd + W_dd) / V after the thermostat
        for (int d = 0; d < 3; ++d) e.ens[13 + d] += (2.0 * l2 * red[1 + d][0] + e.ens[3 + 4 * d]) / e.volume;
    }
}

__global__ __launch_bounds__(BLOCK) void k_ens_scale(EnsArgs e) {
    if (e.status[0] & FREEZE_MASK) return;
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= e.n) return;
    const float lam = (float)e.ens[12];
    for (int b = 0; b < 3; ++b) e.v[(size_t)b * e.n + i] *= lam;
}

__global__ void k_ens_clear(double *ens) {
    if (threadIdx.x < ENS_DOUBLES) ens[threadIdx.x] = 0.0;
}

hipError_t launch_ensemble_clear(double *ens, hipStream_t s) {
    hipLaunchKernelGGL(k_ens_clear, dim3(1), dim3(64), 0, s, ens);
    return hipGetLastError();
}

hipError_t launch_ensemble_step(const EnsArgs &e, hipStream_t s) {
    if (e.n == 0) return hipSuccess;
    const int nb = (e.n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_ens_reduce, dim3(1), dim3(BLOCK), 0, s, e);
    if (e.n_groups > 0)
        hipLaunchKernelGGL(k_con_project, dim3((e.n_groups + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, e, 1);
    hipLaunchKernelGGL(k_ens_finish, dim3(nb), dim3(BLOCK), 0, s, e);
    hipLaunchKernelGGL(k_ens_thermo, dim3(1), dim3(BLOCK), 0, s, e);
    if (e.thermostat) hipLaunchKernelGGL(k_ens_scale, dim3(nb), dim3(BLOCK), 0, s, e);
    return hipGetLastError();
}

}  // namespace nep
