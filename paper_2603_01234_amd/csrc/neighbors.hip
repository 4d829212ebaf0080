// Cell-list neighbour build for the NEP path (the paper only asks for the
// neighbours "within a cutoff distance", Sec. II.A; pair-specific cutoffs as
// for the mixed-resolution model, Sec. II.C.2).
//
// Steps, all on the caller's stream:
//   1. bin:     cell index per bead, per-cell counts (integer atomics), status
//               checks (non-finite, periodic coordinate outside [0, L))
//   2. scan:    exclusive prefix sum of the counts -> cell start offsets
//   3. fill:    scatter bead indices into their cells, then sort every cell
//               by index so the cell contents do not depend on atomic order
//   4. rows:    one thread per bead walks the (2m+1)^3 neighbour cells in a
//               fixed order and applies the exact float32 predicate; angular
//               candidates are written from the front of the row, the others
//               from the back and then moved behind them
//   5. reverse: for every angular entry, the slot of the mirrored entry
#include "nep_internal.h"

namespace nep {

__global__ void k_nb_clear(int ncell, int32_t *cell_count, int32_t *status, int clear_status) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int c = t; c < ncell; c += gridDim.x * blockDim.x) cell_count[c] = 0;
    if (clear_status && t < 4) status[t] = 0;
}

hipError_t launch_clear_status(int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_nb_clear, dim3(1), dim3(64), 0, s, 0, (int32_t *)nullptr, status, 1);
    return hipGetLastError();
}

__device__ __forceinline__ int cell_coord(float x, float inv_cs, int nc) {
    float f = floorf(__fmul_rn(x, inv_cs));
    int k = (int)fminf(fmaxf(f, -1.0f), (float)nc);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

// periodic wrap into [0, L) in float32; a result that rounds to L becomes 0
__device__ __forceinline__ float wrap_coord(float x, float L) {
    float w = x - L * floorf(x / L);
    if (w >= L) w -= L;
    if (w < 0.0f) w += L;
    if (!(w >= 0.0f && w < L)) w = 0.0f;
    return w;
}

__global__ void k_nb_bin(NbArgs a) {
    if (!a.clear_status && (a.status[0] & FREEZE_MASK)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    float p[3] = {a.x[i], a.y[i], a.z[i]};
    if (a.wrap) {
        float *dst[3] = {a.x_mut, a.y_mut, a.z_mut};
        for (int d = 0; d < 3; ++d)
            if (a.pbc[d] && isfinite(p[d])) {
                p[d] = wrap_coord(p[d], a.box[d]);
                dst[d][i] = p[d];
            }
    }
    int flags = 0;
    int c[3];
    for (int d = 0; d < 3; ++d) {
        if (!isfinite(p[d])) { flags |= NEP_FLAG_NONFINITE; p[d] = 0.0f; }
        if (a.pbc[d] && !(p[d] >= 0.0f && p[d] < a.box[d])) flags |= NEP_FLAG_OUTSIDE_BOX;
        c[d] = cell_coord(p[d], a.inv_cs[d], a.nc[d]);
    }
    int t = a.type[i];
    if (t >= a.T) { flags |= NEP_FLAG_BAD_TYPE; t = a.T - 1; }
    if (flags) atomicOr(&a.status[0], flags);
    int cid = (c[2] * a.nc[1] + c[1]) * a.nc[0] + c[0];
    a.cell_id[i] = cid;
    atomicAdd(&a.cell_count[cid], 1);
    a.pos4[i] = make_float4(p[0], p[1], p[2], (float)t);
    a.ref[i] = p[0];
    a.ref[a.n + i] = p[1];
    a.ref[2 * a.n + i] = p[2];
}

// Exclusive scan, three phases.  Block b scans 1024 counts; one block then
// scans the block totals serially in chunks; a last pass adds the offsets.
constexpr int SCAN_B = 1024;

__global__ void k_scan_local(const int32_t *in, int32_t *out, int32_t *block_sums, int n) {
    __shared__ int32_t s[SCAN_B];
    int base = blockIdx.x * SCAN_B;
    int t = threadIdx.x;
    for (int k = t; k < SCAN_B; k += blockDim.x) s[k] = (base + k < n) ? in[base + k] : 0;
    __syncthreads();
    // Hillis-Steele inclusive scan over the block
    for (int off = 1; off < SCAN_B; off <<= 1) {
        int32_t v[SCAN_B / BLOCK];
        for (int q = 0; q < SCAN_B / BLOCK; ++q) {
            int k = t + q * BLOCK;
            v[q] = (k >= off) ? s[k - off] : 0;
        }
        __syncthreads();
        for (int q = 0; q < SCAN_B / BLOCK; ++q) s[t + q * BLOCK] += v[q];
        __syncthreads();
    }
    for (int k = t; k < SCAN_B; k += blockDim.x)
        if (base + k < n) out[base + k] = s[k] - ((base + k < n) ? in[base + k] : 0);
    if (t == 0) block_sums[blockIdx.x] = s[SCAN_B - 1];
}

__global__ void k_scan_blocks(int32_t *block_sums, int nb, int32_t *total_out) {
    if (threadIdx.x != 0) return;
    int32_t run = 0;
    for (int b = 0; b < nb; ++b) {
        int32_t v = block_sums[b];
        block_sums[b] = run;
        run += v;
    }
    *total_out = run;
}

__global__ void k_scan_add(int32_t *out, int32_t *cursor, const int32_t *block_sums, int n) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t v = out[k] + block_sums[k / SCAN_B];
    out[k] = v;
    cursor[k] = v;
}

__global__ void k_nb_fill(NbArgs a) {
    if (!a.clear_status && (a.status[0] & FREEZE_MASK)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    int slot = atomicAdd(&a.cell_cursor[a.cell_id[i]], 1);
    a.cell_list[slot] = i;
}

__global__ void k_nb_sort_cells(NbArgs a) {
    if (!a.clear_status && (a.status[0] & FREEZE_MASK)) return;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    int s = a.cell_start[c], e = s + a.cell_count[c];
    for (int p = s + 1; p < e; ++p) {  // insertion sort by bead index
        int v = a.cell_list[p];
        int q = p - 1;
        while (q >= s && a.cell_list[q] > v) {
            a.cell_list[q + 1] = a.cell_list[q];
            --q;
        }
        a.cell_list[q + 1] = v;
    }
}

__global__ __launch_bounds__(BLOCK) void k_nb_rows(NbArgs a) {
    if (!a.clear_status && (a.status[0] & FREEZE_MASK)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int n = a.n;
    float4 pi = a.pos4[i];
    int ti = (int)pi.w;
    int c0[3];
    c0[0] = cell_coord(pi.x, a.inv_cs[0], a.nc[0]);
    c0[1] = cell_coord(pi.y, a.inv_cs[1], a.nc[1]);
    c0[2] = cell_coord(pi.z, a.inv_cs[2], a.nc[2]);
    int na = 0, nb = 0;  // angular from the front, radial-only from the back
    int flags = 0;
    for (int dz = -a.m[2]; dz <= a.m[2]; ++dz) {
        int kz = c0[2] + dz, iz = 0;
        if (a.pbc[2]) { iz = (kz >= 0) ? kz / a.nc[2] : -((-kz + a.nc[2] - 1) / a.nc[2]); kz -= iz * a.nc[2]; }
        else if (kz < 0 || kz >= a.nc[2]) continue;
        for (int dy = -a.m[1]; dy <= a.m[1]; ++dy) {
            int ky = c0[1] + dy, iy = 0;
            if (a.pbc[1]) { iy = (ky >= 0) ? ky / a.nc[1] : -((-ky + a.nc[1] - 1) / a.nc[1]); ky -= iy * a.nc[1]; }
            else if (ky < 0 || ky >= a.nc[1]) continue;
            for (int dx = -a.m[0]; dx <= a.m[0]; ++dx) {
                int kx = c0[0] + dx, ix = 0;
                if (a.pbc[0]) { ix = (kx >= 0) ? kx / a.nc[0] : -((-kx + a.nc[0] - 1) / a.nc[0]); kx -= ix * a.nc[0]; }
                else if (kx < 0 || kx >= a.nc[0]) continue;
                if (ix < -2 || ix > 2 || iy < -2 || iy > 2 || iz < -2 || iz > 2) { flags |= NEP_FLAG_IMAGE_RANGE; continue; }
                // s = fl(n L), exact predicate with every operation rounded separately
                float sx = __fmul_rn((float)ix, a.box[0]);
                float sy = __fmul_rn((float)iy, a.box[1]);
                float sz = __fmul_rn((float)iz, a.box[2]);
                bool zero_shift = (ix == 0 && iy == 0 && iz == 0);
                uint32_t code = (uint32_t)((ix + 2) + 5 * (iy + 2) + 25 * (iz + 2));
                int cid = (kz * a.nc[1] + ky) * a.nc[0] + kx;
                int s = a.cell_start[cid], e = s + a.cell_count[cid];
                for (int q = s; q < e; ++q) {
                    int j = a.cell_list[q];
                    if (j == i && zero_shift) continue;
                    float4 pj = a.pos4[j];
                    float ddx = __fsub_rn(__fadd_rn(pj.x, sx), pi.x);
                    float ddy = __fsub_rn(__fadd_rn(pj.y, sy), pi.y);
                    float ddz = __fsub_rn(__fadd_rn(pj.z, sz), pi.z);
                    float d2 = __fadd_rn(__fadd_rn(__fmul_rn(ddx, ddx), __fmul_rn(ddy, ddy)),
                                         __fmul_rn(ddz, ddz));
                    int tp = ti * a.T + (int)pj.w;
                    if (!(d2 < a.list2R[tp])) continue;
                    if (d2 == 0.0f) flags |= NEP_FLAG_OVERLAP;
                    uint32_t entry = (uint32_t)j | (code << CODE_SHIFT);
                    if (d2 < a.list2A[tp]) {
                        if (na < a.cap_A && na + nb < a.cap) a.nbr[(size_t)na * n + i] = entry;
                        ++na;
                    } else {
                        if (na + nb < a.cap) a.nbr[(size_t)(a.cap - 1 - nb) * n + i] = entry;
                        ++nb;
                    }
                }
            }
        }
    }
    int total = na + nb;
    if (na > a.cap_A) flags |= NEP_FLAG_OVERFLOW_A;
    if (total > a.cap) flags |= NEP_FLAG_OVERFLOW_R;
    if (flags) atomicOr(&a.status[0], flags);
    if (flags & (NEP_FLAG_OVERFLOW_A | NEP_FLAG_OVERFLOW_R)) {
        atomicMax(&a.status[1], total);
        atomicMax(&a.status[2], na);
        a.cnt[i] = 0;
        a.cnt[n + i] = 0;
        return;
    }
    // move the radial-only entries (stored at slots cap-nb .. cap-1) to slots
    // na .. na+nb-1; the source never lies below the destination, so copying
    // upwards reads every source before it is overwritten
    for (int k = 0; k < nb; ++k)
        a.nbr[(size_t)(na + k) * n + i] = a.nbr[(size_t)(a.cap - nb + k) * n + i];
    a.cnt[i] = total;
    a.cnt[n + i] = na;
    atomicMax(&a.status[1], total);
    atomicMax(&a.status[2], na);
}

__global__ __launch_bounds__(BLOCK) void k_nb_reverse(NbArgs a) {
    if (!a.clear_status && (a.status[0] & FREEZE_MASK)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int n = a.n;
    int na = a.cnt[n + i];
    for (int p = 0; p < na; ++p) {
        uint32_t e = a.nbr[(size_t)p * n + i];
        int j = (int)(e & J_MASK);
        uint32_t code = e >> CODE_SHIFT;
        uint32_t want = (uint32_t)i | ((124u - code) << CODE_SHIFT);
        int nj = a.cnt[n + j];
        int found = -1;
        for (int q = 0; q < nj; ++q)
            if (a.nbr[(size_t)q * n + j] == want) { found = q; break; }
        a.rev[(size_t)p * n + i] = found < 0 ? -1 : (int32_t)((size_t)found * n + j);
    }
}

hipError_t launch_build(const NbArgs &a, hipStream_t s) {
    int nbk = (a.n + BLOCK - 1) / BLOCK;
    int cbk = (a.ncell + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_nb_clear, dim3(cbk > 0 ? (cbk < 4096 ? cbk : 4096) : 1), dim3(BLOCK), 0, s,
                       a.ncell, a.cell_count, a.status, a.clear_status);
    if (a.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_nb_bin, dim3(nbk), dim3(BLOCK), 0, s, a);
    int sb = (a.ncell + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_local, dim3(sb), dim3(BLOCK), 0, s, a.cell_count, a.cell_start, a.scan_tmp, a.ncell);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(64), 0, s, a.scan_tmp, sb, a.cell_start + a.ncell);
    hipLaunchKernelGGL(k_scan_add, dim3(cbk), dim3(BLOCK), 0, s, a.cell_start, a.cell_cursor, a.scan_tmp, a.ncell);
    hipLaunchKernelGGL(k_nb_fill, dim3(nbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_sort_cells, dim3(cbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_rows, dim3(nbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_reverse, dim3(nbk), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace nep
