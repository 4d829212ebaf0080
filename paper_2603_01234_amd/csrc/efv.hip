// NEP energy / force / virial kernels (paper Sec. II.A, Eqs. 2-8; forces from
// E = sum_i U_i; per-site virial of Eq. 15, total of Eq. 16).
//
// k_efv_main: one thread per bead ("centre"), 256 beads per workgroup in a
// cost order written by the build; k_efv_gather: four lanes per bead.  Both
// with an XCD-aware tile map.
//
// k_efv_main    pass 1: loop over the bead's list; radial sums
//                 S_0 = sum hfc,  S_k = sum hfc T_k(x)        (hfc = f_c / 2)
//               so that q_n = c'_n0 S_0 + sum_{k>=1} c_nk S_k with
//               c'_n0 = c_n0 + sum_k c_nk (Eq. 6-7 rearranged: f_k = hfc (T_k + 1));
//               angular sums A_{n,lm} = sum_j g_n(r) P_lm(u) with real solid
//               harmonics, q_nl = sum_m N2_lm A_{n,lm}^2 (equal to Eq. 4).
//               network (Eq. 2) and dU/dq; radial back-propagation
//               coefficients beta_k = sum_n dU/dq_n c_nk stored per bead;
//               pass 2 over the angular candidates: angular part of
//               dU_i/dr_ij into the slot where j lists i (reverse index),
//               and their sum.
// k_efv_gather  F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji):
//               radial part of both terms from the pair geometry and the two
//               beads' beta vectors (no pair buffer); angular dU_j/dr_ji read
//               coalesced from the bead's own slots; per-site virial
//               W_i = sum_j r_ij (x) dU_j/dr_ji; fixed-order block sums of U,
//               W and (for MD) the kinetic energy; optional second half-kick.
// k_reduce      fixed-order FP64 reduction of the block sums.
#include "efv_device.h"

namespace nep {

// positions and (range-clamped) type packed for the neighbour gathers
__global__ void k_pack(int n, int T, const float *__restrict__ x, const float *__restrict__ y,
                       const float *__restrict__ z, const uint8_t *__restrict__ type,
                       float4 *__restrict__ pos4) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos4[i] = make_float4(x[i], y[i], z[i], (float)min((int)type[i], T - 1));
}

hipError_t launch_pack(int n, int T, const float *x, const float *y, const float *z, const uint8_t *type,
                       float4 *pos4, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, n, T, x, y, z, type, pos4);
    return hipGetLastError();
}

template <int NT, int HP, bool MF>
__global__ __launch_bounds__(BLOCK, 2) void k_efv_main(EfvArgs a) {
    extern __shared__ float smem[];
    if constexpr (MF) {
        // the network on the matrix cores: W0 staged once per workgroup; every
        // lane stays to the end (lanes past the system's end with a dummy bead)
        float *w0s = smem;
        mf_stage_w0<HP>(a.ann, w0s);
        __syncthreads();
        if (a.freeze && (a.freeze[0] & FREEZE_MASK)) return;
        const int tile = xcd_tile(blockIdx.x, gridDim.x);
        const int t = tile * BLOCK + threadIdx.x;
        const bool valid = t < a.n;
        int i = valid ? (a.order ? a.order[t] : t) : 0;
        if ((unsigned)i >= (unsigned)a.n) i = valid ? t : 0;
        float *wl = smem + MF_WROWS * (HP + 1) + (threadIdx.x >> 6) * (64 * mf_stride<HP>() + 64);
        main_bead<1, HP, true>(a, a.cut, (const_fp)a.tab, i, valid, w0s, wl);
        return;
    }
    table_ptr<NT> TB;
    if constexpr (NT > 1) {
        // per-pair type indices vary across lanes: stage the pair tables in LDS
        const int nt = NT * NT * TAB_PER_PAIR;
        for (int k = threadIdx.x; k < nt; k += BLOCK) smem[k] = a.tab[k];
        __syncthreads();
        TB = smem;
    } else {
        // one type: every table address is wave-uniform (scalar loads)
        TB = (const_fp)a.tab;
    }
    if (a.freeze && (a.freeze[0] & FREEZE_MASK)) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = tile * BLOCK + threadIdx.x;
    if (t >= a.n) return;
    // the lists' own processing order (written by the build with the rows);
    // an out-of-range entry (a caller's buffer never written) is not trusted
    int i = a.order ? a.order[t] : t;
    if ((unsigned)i >= (unsigned)a.n) i = t;
    main_bead<NT, HP>(a, a.cut, TB, i);
}


// GATHER_LANES lanes per bead: lane q takes slots q, q + GATHER_LANES, ... of
// the row (lane 0 also the bead's own angular sum), and the lane sums are
// combined by a shuffle butterfly (more waves in flight for the neighbour
// gathers).  The batched and the served gathers split and add in the same way.
constexpr int GATHER_BEADS = BLOCK / GATHER_LANES;

// MD: 0 plain evaluation, 1 NVE step (second half-kick fused), 2 ensemble
// step (forces with the HNEMD drive when HN, per-bead virial; no kick)
template <int NT, bool VIR, int MD, bool HN>
__global__ __launch_bounds__(BLOCK) void k_efv_gather(GatherArgs a) {
    constexpr int NP = MD == 2 ? NPART : NPART_NVE;
    __shared__ double red[NP][BLOCK / 64];
    if (MD && a.freeze && (a.freeze[0] & FREEZE_MASK)) return;  // uniform over the grid
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = threadIdx.x % GATHER_LANES;
    const int i = tile * GATHER_BEADS + (int)(threadIdx.x / GATHER_LANES);
    const int n = a.n;
    double acc[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) acc[c] = 0.0;
    int nR_in = 0, nA_in = 0;  // pairs inside the interaction cutoffs (work accounting)
    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, W[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) W[c] = 0.0f;
    float4 pi = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int ti = 0;
    if (i < n) {
        pi = a.pos4[i];
        ti = (NT == 1) ? 0 : (int)pi.w;
        gather_bead<NT, VIR>(a, a.cut, i, pi, ti, Fx, Fy, Fz, W, nR_in, nA_in, q, GATHER_LANES);
    }
    // every lane takes part in the exchange
#pragma unroll
    for (int o = 1; o < GATHER_LANES; o <<= 1) {
        Fx += __shfl_xor(Fx, o);
        Fy += __shfl_xor(Fy, o);
        Fz += __shfl_xor(Fz, o);
        if (VIR) {
#pragma unroll
            for (int c = 0; c < 9; ++c) W[c] += __shfl_xor(W[c], o);
        }
        nR_in += __shfl_xor(nR_in, o);
        nA_in += __shfl_xor(nA_in, o);
    }
    if (i < n && q == 0) {
        if (HN) {
            // HNEMD drive W_i^T F_e (its mean is removed by the ensemble kernels)
            float fe[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) fe[b] = W[b] * a.Fe[0] + W[3 + b] * a.Fe[1] + W[6 + b] * a.Fe[2];
            Fx += fe[0];
            Fy += fe[1];
            Fz += fe[2];
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[13 + b] = (double)fe[b];
        }
        a.F[i] = Fx;
        a.F[n + i] = Fy;
        a.F[2 * n + i] = Fz;
        acc[0] = (double)a.U[i];
        acc[11] = (double)nR_in;
        acc[12] = (double)nA_in;
        if (VIR) {
            if (a.W) {
#pragma unroll
                for (int c = 0; c < 9; ++c) a.W[(size_t)c * n + i] = W[c];
            }
#pragma unroll
            for (int c = 0; c < 9; ++c) acc[1 + c] = (double)W[c];
        }
        if (MD == 1) {
            // second half-kick from the half-step velocity; the step's new
            // state (x, v) is committed to the caller's arrays only here, so
            // a step stopped by a failed rebuild leaves the previous one whole
            float k = a.half_dt_accel * a.inv_mass[ti];
            float vx = a.vh[i] + k * Fx;
            float vy = a.vh[n + i] + k * Fy;
            float vz = a.vh[2 * n + i] + k * Fz;
            a.v[i] = vx;
            a.v[n + i] = vy;
            a.v[2 * n + i] = vz;
            a.x[i] = pi.x;
            a.y[i] = pi.y;
            a.z[i] = pi.z;
            acc[10] = 0.5 * (double)a.mass[ti] * ((double)vx * vx + (double)vy * vy + (double)vz * vz) /
                      (double)ACCEL;
        }
    }
    if (!MD && a.top2) {
        // displacement since the build, for the completeness test of the lists
        // (the reduction merges the blocks' pairs)
        float d2 = 0.0f;
        if (i < n && q == 0) {
            const float dx = pi.x - a.ref[i], dy = pi.y - a.ref[n + i], dz = pi.z - a.ref[2 * n + i];
            d2 = dx * dx + dy * dy + dz * dz;
        }
        const float2 t = block_top2(d2, 0.0f);
        if (threadIdx.x == 0) a.top2[tile] = t;
    }
    // fixed-order block sums: a butterfly within each wave (lane 0's result),
    // then the waves in order
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        double v = acc[c];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        if (__lane_id() == 0) red[c][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < NP) {
        double v = red[threadIdx.x][0];
#pragma unroll
        for (int w = 1; w < BLOCK / 64; ++w) v += red[threadIdx.x][w];
        a.partial[(size_t)tile * NPART + threadIdx.x] = v;
    }
}

// The reduction of the block partials (reduce_partials), after the optional
// merge of the gather blocks' displacement pairs for the standalone rebuild
// test.
__global__ void k_reduce(const double *__restrict__ partial, int nblocks, double *E_tot,
                         double *W_tot, double *K_tot, double *E_slot, double *K_slot, double *W_slot,
                         double *counts, const int32_t *status, int32_t *ctrl, int next_gate,
                         const float2 *top2, float skin_gate, float reach, int32_t *skin_status) {
    if (top2) {
        const float2 t = merge_top2(top2, nblocks);
        if (threadIdx.x == 0 && past_skin(t, skin_gate, (1.0f - sigma_of(skin_status[3])) * reach))
            atomicOr(skin_status, NEP_FLAG_SKIN);
    }
    reduce_partials(partial, nblocks, E_tot, W_tot, K_tot, E_slot, K_slot, W_slot, counts, status, ctrl,
                    next_gate);
}

hipError_t launch_reduce(const double *partial, int nblocks, double *E_tot, double *W_tot,
                         double *K_tot, double *E_slot, double *K_slot, double *W_slot, double *counts,
                         const int32_t *status, int32_t *ctrl, int next_gate, const float2 *top2,
                         float skin_gate, float reach, int32_t *skin_status, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLOCK), 0, s, partial, nblocks, E_tot, W_tot, K_tot,
                       E_slot, K_slot, W_slot, counts, status, ctrl, next_gate, top2, skin_gate, reach,
                       skin_status);
    return hipGetLastError();
}

template <int NT, int HP, bool MF = false>
static hipError_t main_t(const EfvArgs &a, size_t lds, hipStream_t s) {
    int nb = (a.n + BLOCK - 1) / BLOCK;
    if constexpr (MF) lds = (size_t)mf_lds_floats<HP>(BLOCK / 64) * sizeof(float);
    hipLaunchKernelGGL((k_efv_main<NT, HP, MF>), dim3(nb), dim3(BLOCK), (NT > 1 || MF) ? lds : 0, s, a);
    return hipGetLastError();
}

template <int NT>
static hipError_t main_nt(int HP, const EfvArgs &a, size_t lds, hipStream_t s) {
    switch (HP) {
        case 8: return main_t<NT, 8>(a, lds, s);
        case 16: return main_t<NT, 16>(a, lds, s);
        case 32: return main_t<NT, 32>(a, lds, s);
        case 64: return main_t<NT, 64>(a, lds, s);
    }
    return hipErrorInvalidValue;
}

bool efv_main_mfma_supported(int T, int HP) { return T == 1 && (HP == 16 || HP == 32 || HP == 64); }

hipError_t launch_efv_main(int T, int HP, const EfvArgs &a, size_t lds, hipStream_t s, bool mfma) {
    if (a.n == 0) return hipSuccess;
    if (mfma) {
        if (!efv_main_mfma_supported(T, HP)) return hipErrorInvalidValue;
        switch (HP) {
            case 16: return main_t<1, 16, true>(a, lds, s);
            case 32: return main_t<1, 32, true>(a, lds, s);
            case 64: return main_t<1, 64, true>(a, lds, s);
        }
    }
    switch (T) {
        case 1: return main_nt<1>(HP, a, lds, s);
        case 2: return main_nt<2>(HP, a, lds, s);
        case 3: return main_nt<3>(HP, a, lds, s);
        case 4: return main_nt<4>(HP, a, lds, s);
    }
    return hipErrorInvalidValue;
}

template <int NT, bool VIR, int MD, bool HN>
static hipError_t gather_t(const GatherArgs &a, hipStream_t s) {
    int nb = (a.n + GATHER_BEADS - 1) / GATHER_BEADS;
    hipLaunchKernelGGL((k_efv_gather<NT, VIR, MD, HN>), dim3(nb), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// built forms: plain with or without the virial, the NVE step (always with
// the virial), the ensemble step with or without the HNEMD drive
template <int NT>
static hipError_t gather_nt(bool vir, int md, bool hn, const GatherArgs &a, hipStream_t s) {
    if (md == 2) return hn ? gather_t<NT, true, 2, true>(a, s) : gather_t<NT, true, 2, false>(a, s);
    if (md == 1) return gather_t<NT, true, 1, false>(a, s);
    return vir ? gather_t<NT, true, 0, false>(a, s) : gather_t<NT, false, 0, false>(a, s);
}

hipError_t launch_efv_gather(int T, bool vir, int md, bool hn, const GatherArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (T) {
        case 1: return gather_nt<1>(vir, md, hn, a, s);
        case 2: return gather_nt<2>(vir, md, hn, a, s);
        case 3: return gather_nt<3>(vir, md, hn, a, s);
        case 4: return gather_nt<4>(vir, md, hn, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace nep
