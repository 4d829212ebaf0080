// Batched energy / force / virial evaluation for the fitness loop: many
// parameter sets (candidates of the evolution strategy, Sec. II.A) over many
// structures, with the loss terms (RMSE of energies and virials per bead and
// of forces per component) reduced on the device.
//
// k_efv_batch is persistent: its workgroups take (candidate, structure) items
// from an atomic counter until the list is exhausted.  One item is one
// complete evaluation of one structure by one workgroup: pack positions,
// fused descriptor / network / angular pass over every bead, barrier, gather
// pass with the residuals against the labels, fixed-order block sums into the
// item's record.  Intermediates live in the workgroup's own slice of the
// workspace, sized for the largest structure.  k_batch_rmse then sums the
// records of each candidate in item order, so the result does not depend on
// which workgroup took which item.
#include "efv_device.h"

namespace nep {

constexpr int REC = 12;  // record per item: E, sum |F - F_ref|^2, W[9], pairs within r_c

template <int NT, int HP, int BS>
__global__ __launch_bounds__(BS, 2) void k_efv_batch(BatchArgs b) {
    extern __shared__ float smem[];  // pair tables of the current candidate (several types)
    __shared__ double red[REC][BS];
    __shared__ int s_item;
    char *base = b.scratch + (size_t)blockIdx.x * b.scratch_stride;
    float4 *pos4 = (float4 *)base;
    float4 *fown = pos4 + b.nmax;
    float4 *bvec = fown + b.nmax;
    float4 *angbuf = bvec + (size_t)b.nmax * NT * 3;
    float *U = (float *)(angbuf + (size_t)b.nmax * b.capAmax);
    int cur_model = -1;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(b.counter, 1);
        __syncthreads();
        // uniform over the workgroup: keep the item and everything loaded from
        // it in scalar registers
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= b.n_items) break;  // every workgroup ends here once the list is taken
        const int4 w = b.items[it];  // model, system, index in the caller's list
        const SysDesc &sd = b.sys[w.y];
        const ModelDesc &md = b.mod[w.x];
        // the candidate's tables, in scalar registers (the item is uniform)
        const float *tab = uniform_ptr(md.tab);
        const float *ann = uniform_ptr(md.ann);
        const int n = sd.n;
        table_ptr<NT> TB;
        if constexpr (NT > 1) {
            if (w.x != cur_model) {
                for (int k = threadIdx.x; k < NT * NT * TAB_PER_PAIR; k += BS) smem[k] = tab[k];
                cur_model = w.x;
            }
            TB = smem;
        } else {
            TB = (const_fp)tab;
        }
        for (int i = threadIdx.x; i < n; i += BS)
            pos4[i] = make_float4(sd.x[i], sd.y[i], sd.z[i], (float)min((int)sd.type[i], NT - 1));
        __syncthreads();

        EfvArgs a{};
        a.n = n;
        a.box[0] = sd.box[0];
        a.box[1] = sd.box[1];
        a.box[2] = sd.box[2];
        a.pos4 = pos4;
        a.nbr = sd.nbr;
        a.rev = sd.rev;
        a.cnt = sd.cnt;
        a.tab = tab;
        a.ann = ann;
        a.U = U;
        a.bvec = bvec;
        a.angbuf = angbuf;
        a.fown = fown;
        for (int i0 = 0; i0 < n; i0 += BS) {
            const int i = i0 + threadIdx.x;
            if (i < n) main_bead<NT, HP>(a, b.cut, TB, i);
        }
        __syncthreads();

        GatherArgs g{};
        g.n = n;
        g.box[0] = sd.box[0];
        g.box[1] = sd.box[1];
        g.box[2] = sd.box[2];
        g.pos4 = pos4;
        g.nbr = sd.nbr;
        g.cnt = sd.cnt;
        g.bvec = bvec;
        g.angbuf = angbuf;
        g.fown = fown;
        double acc[REC];
#pragma unroll
        for (int c = 0; c < REC; ++c) acc[c] = 0.0;
        const double *Fr = b.F_ref ? b.F_ref + (size_t)sd.label_off * 3 : nullptr;
        float *Fo = b.F_out ? b.F_out + (size_t)b.F_off[w.z] * 3 : nullptr;
        // GATHER_LANES lanes per bead, combined as the single-system gather does
        for (int i0 = 0; i0 < n; i0 += BS / GATHER_LANES) {
            const int i = i0 + (int)(threadIdx.x / GATHER_LANES);
            const int q = threadIdx.x % GATHER_LANES;
            float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, W[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) W[c] = 0.0f;
            int nR = 0, nA = 0;
            if (i < n) {
                const float4 pi = pos4[i];
                const int ti = (NT == 1) ? 0 : (int)pi.w;
                gather_bead<NT, true>(g, b.cut, i, pi, ti, Fx, Fy, Fz, W, nR, nA, q, GATHER_LANES);
            }
            // every lane takes part in the exchange
#pragma unroll
            for (int o = 1; o < GATHER_LANES; o <<= 1) {
                Fx += __shfl_xor(Fx, o);
                Fy += __shfl_xor(Fy, o);
                Fz += __shfl_xor(Fz, o);
#pragma unroll
                for (int c = 0; c < 9; ++c) W[c] += __shfl_xor(W[c], o);
                nR += __shfl_xor(nR, o);
            }
            if (i < n && q == 0) {
                acc[0] += (double)U[i];
                if (Fr) {
                    const double dx = (double)Fx - Fr[3 * i], dy = (double)Fy - Fr[3 * i + 1],
                                 dz = (double)Fz - Fr[3 * i + 2];
                    acc[1] += dx * dx + dy * dy + dz * dz;
                }
#pragma unroll
                for (int c = 0; c < 9; ++c) acc[2 + c] += (double)W[c];
                acc[11] += (double)nR;
                if (Fo) {
                    Fo[3 * i] = Fx;
                    Fo[3 * i + 1] = Fy;
                    Fo[3 * i + 2] = Fz;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < REC; ++c) red[c][threadIdx.x] = acc[c];
        __syncthreads();
        for (int s = BS / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
#pragma unroll
                for (int c = 0; c < REC; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x < REC) b.records[(size_t)w.z * REC + threadIdx.x] = red[threadIdx.x][0];
        // the next item overwrites the scratch and the reduction buffer
        __syncthreads();
    }
}

__global__ void k_batch_reset(int *counter) {
    if (threadIdx.x == 0) *counter = 0;
}

// One workgroup per candidate: its items in list order, fixed-order sums.
//   RMSE_E = sqrt(mean_s ((E_s - E_s^ref) / N_s)^2)
//   RMSE_F = sqrt(sum |F - F^ref|^2 / (3 sum_s N_s))
//   RMSE_W = sqrt(mean_s mean_6 ((W_s - W_s^ref) / N_s)^2)  (xx yy zz xy yz xz)
__global__ __launch_bounds__(BLOCK) void k_batch_rmse(int n_items, const int4 *list, const SysDesc *sys,
                                                      const double *records, const double *E_ref,
                                                      const double *W_ref, double *rmse, double *item_out) {
    __shared__ double red[5][BLOCK];
    const int m = blockIdx.x;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // E, F, W terms, structures, force components
    for (int it = threadIdx.x; it < n_items; it += BLOCK) {
        const int4 w = list[it];
        const double *r = records + (size_t)it * REC;
        if (m == 0 && item_out) {
            item_out[(size_t)it * 10] = r[0];
            for (int c = 0; c < 9; ++c) item_out[(size_t)it * 10 + 1 + c] = r[2 + c];
        }
        if (w.x != m || !rmse) continue;
        const double N = (double)sys[w.y].n;
        if (N == 0.0) continue;
        const double eE = (r[0] - E_ref[w.y]) / N;
        acc[0] += eE * eE;
        acc[1] += r[1];
        const int comp[6] = {0, 4, 8, 1, 5, 2};
        for (int c = 0; c < 6; ++c) {
            const double d = (r[2 + comp[c]] - W_ref[(size_t)w.y * 9 + comp[c]]) / N;
            acc[2] += d * d;
        }
        acc[3] += 1.0;
        acc[4] += 3.0 * N;
    }
    for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && rmse) {
        const double ns = red[3][0], nf = red[4][0];
        rmse[m * 3 + 0] = ns > 0.0 ? sqrt(red[0][0] / ns) : 0.0;
        rmse[m * 3 + 1] = nf > 0.0 ? sqrt(red[1][0] / nf) : 0.0;
        rmse[m * 3 + 2] = ns > 0.0 ? sqrt(red[2][0] / (6.0 * ns)) : 0.0;
    }
}

template <int NT, int HP, int BS>
static hipError_t batch_t(const BatchArgs &b, int grid, hipStream_t s) {
    const size_t lds = NT > 1 ? (size_t)NT * NT * TAB_PER_PAIR * sizeof(float) : 0;
    hipLaunchKernelGGL((k_efv_batch<NT, HP, BS>), dim3(grid), dim3(BS), lds, s, b);
    return hipGetLastError();
}

template <int NT, int HP, int BS>
static int occupancy_t() {
    int nb = 0;
    const size_t lds = NT > 1 ? (size_t)NT * NT * TAB_PER_PAIR * sizeof(float) : 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_efv_batch<NT, HP, BS>, BS, lds) != hipSuccess)
        return 0;
    return nb;
}

#define NEP_BATCH_DISPATCH(FN, ...)                                                              \
    switch (T * 1000 + HP * 10 + (BS == 64 ? 0 : BS == 128 ? 1 : 2)) {                          \
        case 1080: return FN<1, 8, 64>(__VA_ARGS__);                                             \
        case 1081: return FN<1, 8, 128>(__VA_ARGS__);                                            \
        case 1082: return FN<1, 8, 256>(__VA_ARGS__);                                            \
        case 1160: return FN<1, 16, 64>(__VA_ARGS__);                                            \
        case 1161: return FN<1, 16, 128>(__VA_ARGS__);                                           \
        case 1162: return FN<1, 16, 256>(__VA_ARGS__);                                           \
        case 1320: return FN<1, 32, 64>(__VA_ARGS__);                                            \
        case 1321: return FN<1, 32, 128>(__VA_ARGS__);                                           \
        case 1322: return FN<1, 32, 256>(__VA_ARGS__);                                           \
        case 1640: return FN<1, 64, 64>(__VA_ARGS__);                                            \
        case 1641: return FN<1, 64, 128>(__VA_ARGS__);                                           \
        case 1642: return FN<1, 64, 256>(__VA_ARGS__);                                           \
        case 2080: return FN<2, 8, 64>(__VA_ARGS__);                                             \
        case 2081: return FN<2, 8, 128>(__VA_ARGS__);                                            \
        case 2082: return FN<2, 8, 256>(__VA_ARGS__);                                            \
        case 2160: return FN<2, 16, 64>(__VA_ARGS__);                                            \
        case 2161: return FN<2, 16, 128>(__VA_ARGS__);                                           \
        case 2162: return FN<2, 16, 256>(__VA_ARGS__);                                           \
        case 2320: return FN<2, 32, 64>(__VA_ARGS__);                                            \
        case 2321: return FN<2, 32, 128>(__VA_ARGS__);                                           \
        case 2322: return FN<2, 32, 256>(__VA_ARGS__);                                           \
        case 2640: return FN<2, 64, 64>(__VA_ARGS__);                                            \
        case 2641: return FN<2, 64, 128>(__VA_ARGS__);                                           \
        case 2642: return FN<2, 64, 256>(__VA_ARGS__);                                           \
    }

hipError_t launch_efv_batch(int T, int HP, int BS, const BatchArgs &b, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, b.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.n_items == 0) return hipSuccess;
    NEP_BATCH_DISPATCH(batch_t, b, grid, s)
    return hipErrorInvalidValue;
}

int batch_occupancy(int T, int HP, int BS) {
    NEP_BATCH_DISPATCH(occupancy_t)
    return 0;
}

hipError_t launch_batch_rmse(int n_models, int n_items, const int4 *list, const SysDesc *sys,
                             const double *records, const double *E_ref, const double *W_ref, double *rmse,
                             double *item_out, hipStream_t s) {
    if (n_models == 0 || (!rmse && !item_out)) return hipSuccess;
    hipLaunchKernelGGL(k_batch_rmse, dim3(n_models), dim3(BLOCK), 0, s, n_items, list, sys, records, E_ref,
                       W_ref, rmse, item_out);
    return hipGetLastError();
}

}  // namespace nep
