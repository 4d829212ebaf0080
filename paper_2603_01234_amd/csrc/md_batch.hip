// One velocity-Verlet step for many independent replicas (the served form):
// every kernel runs once over the tiles of all active replicas.  A workgroup
// finds its replica by a search over the replicas' first tiles; each replica
// keeps its own state, lists and workspace, so a replica's results do not
// depend on which others share the step.
#include "efv_device.h"

namespace nep {

__device__ __forceinline__ int replica_of(const MdBatchArgs &b, int tile) {
    int lo = 0, hi = b.n_rep - 1;  // last replica whose first tile is <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.tile_start[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(BLOCK) void k_kick_drift_batch(MdBatchArgs b) {
    const int r = replica_of(b, blockIdx.x);
    const RepDesc &d = b.rep[r];
    if (d.status[0] & FREEZE_MASK) return;  // uniform over the replica's workgroups
    const int tile = blockIdx.x - b.tile_start[r];
    const int i = tile * BLOCK + threadIdx.x;
    float d2 = 0.0f;
    if (i < d.n) {
        const int t = min((int)d.type[i], b.T - 1);
        const float k = b.half_dt_accel * b.inv_mass[t];
        d2 = kick_drift_bead(i, d.n, t, k, b.dt, 1.0f, 1.0f, 1.0f, d.x, d.y, d.z, d.v, d.vh, d.F, d.pos4, d.ref);
    }
    const float2 t = block_top2(d2, 0.0f);
    if (threadIdx.x == 0) d.top2[tile] = t;
}

// one workgroup per replica: the rebuild test over its tiles' pairs (the same
// test over the same beads as the single-replica step)
__global__ __launch_bounds__(BLOCK) void k_gate_batch(MdBatchArgs b) {
    const int r = blockIdx.x;
    const RepDesc &d = b.rep[r];
    if (d.status[0] & FREEZE_MASK) return;
    const float2 t = merge_top2(d.top2, b.tile_start[r + 1] - b.tile_start[r]);
    if (threadIdx.x == 0) {
        // no strain here: sigma only carries over from a compressive run
        const float sig = sigma_of(d.status[3]);
        if (past_skin(t, d.skin_gate, (1.0f - sig) * d.reach)) b.gate[r] = 1;
        if (b.gate[r]) d.status[3] = SIGMA_ONE;
    }
}

template <int NT, int HP>
__global__ __launch_bounds__(BLOCK, 2) void k_efv_main_batch(MdBatchArgs b) {
    extern __shared__ float smem[];
    table_ptr<NT> TB;
    if constexpr (NT > 1) {
        for (int k = threadIdx.x; k < NT * NT * TAB_PER_PAIR; k += BLOCK) smem[k] = b.tab[k];
        __syncthreads();
        TB = smem;
    } else {
        TB = (const_fp)b.tab;
    }
    const int r = replica_of(b, blockIdx.x);
    const RepDesc &d = b.rep[r];
    if (d.status[0] & FREEZE_MASK) return;
    const int t = (blockIdx.x - b.tile_start[r]) * BLOCK + threadIdx.x;
    if (t >= d.n) return;
    // the lists' processing order (beads of similar cost side by side); an
    // out-of-range entry (a buffer never written) is not trusted
    int i = d.order ? d.order[t] : t;
    if ((unsigned)i >= (unsigned)d.n) i = t;
    EfvArgs a{};
    a.n = d.n;
    a.box[0] = d.box[0];
    a.box[1] = d.box[1];
    a.box[2] = d.box[2];
    a.pos4 = d.pos4;
    a.nbr = d.nbr;
    a.rev = d.rev;
    a.cnt = d.cnt;
    a.tab = b.tab;
    a.ann = b.ann;
    a.U = d.U;
    a.bvec = d.bvec;
    a.angbuf = d.angbuf;
    a.fown = d.fown;
    main_bead<NT, HP>(a, b.cut, TB, i);
}

// Forces, second half-kick, commit of x and v, and per-tile sums of the
// potential and kinetic energy into the replica's partial buffer.
// GATHER_LANES lanes per bead (combined as in the single-system gather), so a
// workgroup of GATHER_LANES * BLOCK threads covers one tile of BLOCK beads.
template <int NT>
__global__ __launch_bounds__(GATHER_LANES * BLOCK) void k_efv_gather_batch(MdBatchArgs b) {
    __shared__ double red[2][GATHER_LANES * BLOCK];
    const int r = replica_of(b, blockIdx.x);
    const RepDesc &d = b.rep[r];
    if (d.status[0] & FREEZE_MASK) return;  // uniform over the workgroup
    const int tile = blockIdx.x - b.tile_start[r];
    const int q = threadIdx.x % GATHER_LANES;
    const int i = tile * BLOCK + (int)(threadIdx.x / GATHER_LANES);
    const int n = d.n;
    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
    float4 pi = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int ti = 0;
    if (i < n) {
        GatherArgs g{};
        g.n = n;
        g.box[0] = d.box[0];
        g.box[1] = d.box[1];
        g.box[2] = d.box[2];
        g.pos4 = d.pos4;
        g.nbr = d.nbr;
        g.cnt = d.cnt;
        g.bvec = d.bvec;
        g.angbuf = d.angbuf;
        g.fown = d.fown;
        pi = d.pos4[i];
        ti = (NT == 1) ? 0 : (int)pi.w;
        float W[9];
        int nR = 0, nA = 0;
        gather_bead<NT, false>(g, b.cut, i, pi, ti, Fx, Fy, Fz, W, nR, nA, q, GATHER_LANES);
    }
    // every lane takes part in the exchange
#pragma unroll
    for (int o = 1; o < GATHER_LANES; o <<= 1) {
        Fx += __shfl_xor(Fx, o);
        Fy += __shfl_xor(Fy, o);
        Fz += __shfl_xor(Fz, o);
    }
    double eU = 0.0, eK = 0.0;
    if (i < n && q == 0) {
        d.F[i] = Fx;
        d.F[n + i] = Fy;
        d.F[2 * n + i] = Fz;
        const float k = b.half_dt_accel * b.inv_mass[ti];
        const float vx = d.vh[i] + k * Fx;
        const float vy = d.vh[n + i] + k * Fy;
        const float vz = d.vh[2 * n + i] + k * Fz;
        d.v[i] = vx;
        d.v[n + i] = vy;
        d.v[2 * n + i] = vz;
        d.x[i] = pi.x;
        d.y[i] = pi.y;
        d.z[i] = pi.z;
        eU = (double)d.U[i];
        eK = 0.5 * (double)b.mass[ti] * ((double)vx * vx + (double)vy * vy + (double)vz * vz) / (double)ACCEL;
    }
    red[0][threadIdx.x] = eU;
    red[1][threadIdx.x] = eK;
    __syncthreads();
    for (int s = GATHER_LANES * BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) d.partial[(size_t)tile * 2 + threadIdx.x] = red[threadIdx.x][0];
}

// one workgroup per replica: fixed-order sums of its tiles, and a copy of the
// replica's status word for the host
__global__ __launch_bounds__(BLOCK) void k_reduce_batch(MdBatchArgs b) {
    __shared__ double red[2][BLOCK];
    const int r = blockIdx.x;
    const RepDesc &d = b.rep[r];
    if (threadIdx.x < 4) b.status_out[4 * r + threadIdx.x] = d.status[threadIdx.x];
    if (d.status[0] & FREEZE_MASK) return;
    const int nt = b.tile_start[r + 1] - b.tile_start[r];
    double e = 0.0, k = 0.0;
    for (int t = threadIdx.x; t < nt; t += BLOCK) {
        e += d.partial[(size_t)t * 2];
        k += d.partial[(size_t)t * 2 + 1];
    }
    red[0][threadIdx.x] = e;
    red[1][threadIdx.x] = k;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (b.E_pot) b.E_pot[r] = red[0][0];
        if (b.E_kin) b.E_kin[r] = red[1][0];
    }
}

hipError_t launch_kick_drift_batch(const MdBatchArgs &b, hipStream_t s) {
    if (b.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_drift_batch, dim3(b.n_tiles), dim3(BLOCK), 0, s, b);
    hipLaunchKernelGGL(k_gate_batch, dim3(b.n_rep), dim3(BLOCK), 0, s, b);
    return hipGetLastError();
}

template <int NT, int HP>
static hipError_t main_batch_t(const MdBatchArgs &b, hipStream_t s) {
    const size_t lds = NT > 1 ? (size_t)NT * NT * TAB_PER_PAIR * sizeof(float) : 0;
    hipLaunchKernelGGL((k_efv_main_batch<NT, HP>), dim3(b.n_tiles), dim3(BLOCK), lds, s, b);
    return hipGetLastError();
}

template <int NT>
static hipError_t main_batch_nt(int HP, const MdBatchArgs &b, hipStream_t s) {
    switch (HP) {
        case 8: return main_batch_t<NT, 8>(b, s);
        case 16: return main_batch_t<NT, 16>(b, s);
        case 32: return main_batch_t<NT, 32>(b, s);
        case 64: return main_batch_t<NT, 64>(b, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_efv_md_batch(int T, int HP, const MdBatchArgs &b, hipStream_t s) {
    // the per-replica sums (and status copies) run even when every replica is empty
    if (b.n_tiles == 0) {
        hipLaunchKernelGGL(k_reduce_batch, dim3(b.n_rep), dim3(BLOCK), 0, s, b);
        return hipGetLastError();
    }
    hipError_t e = hipErrorInvalidValue;
    switch (T) {
        case 1: e = main_batch_nt<1>(HP, b, s); break;
        case 2: e = main_batch_nt<2>(HP, b, s); break;
        case 3: e = main_batch_nt<3>(HP, b, s); break;
        case 4: e = main_batch_nt<4>(HP, b, s); break;
    }
    if (e != hipSuccess) return e;
    switch (T) {
        case 1: hipLaunchKernelGGL(k_efv_gather_batch<1>, dim3(b.n_tiles), dim3(GATHER_LANES * BLOCK), 0, s, b); break;
        case 2: hipLaunchKernelGGL(k_efv_gather_batch<2>, dim3(b.n_tiles), dim3(GATHER_LANES * BLOCK), 0, s, b); break;
        case 3: hipLaunchKernelGGL(k_efv_gather_batch<3>, dim3(b.n_tiles), dim3(GATHER_LANES * BLOCK), 0, s, b); break;
        case 4: hipLaunchKernelGGL(k_efv_gather_batch<4>, dim3(b.n_tiles), dim3(GATHER_LANES * BLOCK), 0, s, b); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_batch, dim3(b.n_rep), dim3(BLOCK), 0, s, b);
    return hipGetLastError();
}

}  // namespace nep
