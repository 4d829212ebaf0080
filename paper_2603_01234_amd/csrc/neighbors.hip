// Cell-list neighbour build for the NEP path (the descriptors run over the
// neighbours inside a cutoff, Sec. II.A; pair-specific cutoffs as for the
// mixed-resolution model, Sec. II.C.2).
//
// Steps, all on the caller's stream:
//   1. bin:     cell index per bead, per-cell counts (integer atomics), status
//               checks (non-finite, periodic coordinate outside [0, L))
//   2. scan:    exclusive prefix sum of the counts -> cell start offsets
//   3. fill:    scatter bead indices into their cells (atomic order), then
//               give every bead its rank by index within its cell, so cell
//               contents and a cell-ordered copy of the positions are in one
//               canonical order whatever the atomics did
//   4. rows:    one thread per bead walks the (2m+1)^3 neighbour cells in a
//               fixed order over the cell-ordered positions and applies the
//               exact float32 predicate; entries go to four stacks of a
//               row-major scratch row by class (angular inside r_c^A, angular
//               shell, radial-only inside r_c^R, radial shell)
//   5. transpose: scratch rows -> slot-major lists in that class order
//   6. reverse: for every angular entry, the mirrored entry is searched among
//               the neighbour's angular entries in its scratch row
#include "nep_internal.h"

// The list predicate is exact only with every float operation rounded on its
// own.  The operations are written here, where contraction into fused
// multiply-adds is switched off; the library's __f*_rn helpers are compiled
// under the default setting and get fused once inlined.
#pragma clang fp contract(off)

namespace nep {

__device__ __forceinline__ float mul_rn(float a, float b) { return a * b; }
__device__ __forceinline__ float add_rn(float a, float b) { return a + b; }
__device__ __forceinline__ float sub_rn(float a, float b) { return a - b; }

// A build inside an MD run is skipped when neither the drift's rebuild test
// nor the schedule asked for one (ctrl[0] == 0), and once the run is frozen
// after a failed build.  The test is uniform over the grid.
__device__ __forceinline__ bool build_off(const int32_t *ctrl, const int32_t *status, int clear_status) {
    if (ctrl && ctrl[0] == 0) return true;
    return !clear_status && (status[0] & FREEZE_MASK);
}
__device__ __forceinline__ bool build_off(const NbArgs &a) { return build_off(a.ctrl, a.status, a.clear_status); }

// Every phase of the build is a body taking its block index and block count,
// so that the same code runs as one kernel per system or as one kernel over
// the blocks of many systems (the served form).
__device__ __forceinline__ void nb_clear_body(int ncell, int32_t *cell_count, int32_t *status, int clear_status,
                                              int32_t *ctrl, int bx, int gx) {
    if (build_off(ctrl, status, clear_status)) return;
    int t = bx * blockDim.x + threadIdx.x;
    for (int c = t; c < ncell; c += gx * blockDim.x) cell_count[c] = 0;
    // a fresh build: no flags, and the lists start uncompressed (sigma = 1)
    if (clear_status && t < 4) status[t] = t == 3 ? SIGMA_ONE : 0;
    if (ctrl && t == 0) ctrl[1] += 1;
}

__global__ void k_nb_clear(int ncell, int32_t *cell_count, int32_t *status, int clear_status, int32_t *ctrl) {
    nb_clear_body(ncell, cell_count, status, clear_status, ctrl, blockIdx.x, gridDim.x);
}

// start of an MD call: flags and maxima cleared, sigma (status[3]) kept, since
// it belongs to the lists, which the call continues from
__global__ void k_md_clear(int32_t *status, int32_t *ctrl, int gate0) {
    int t = threadIdx.x;
    if (t < 3) status[t] = 0;
    if (ctrl && t < 4) ctrl[t] = t == 0 ? gate0 : 0;
}

hipError_t launch_clear_status(int32_t *status, int32_t *ctrl, int gate0, hipStream_t s) {
    hipLaunchKernelGGL(k_md_clear, dim3(1), dim3(64), 0, s, status, ctrl, gate0);
    return hipGetLastError();
}

__device__ __forceinline__ int cell_coord(float x, float inv_cs, int nc) {
    float f = floorf(mul_rn(x, inv_cs));
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

__device__ __forceinline__ void nb_bin_body(const NbArgs &a, int bx) {
    if (build_off(a)) return;
    if (a.skip_clear && a.ctrl && bx == 0 && threadIdx.x == 0) a.ctrl[1] += 1;  // the clear phase's count
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    float p[3];
    if (a.from_pos4) {
        const float4 q = a.pos4[i];
        p[0] = q.x; p[1] = q.y; p[2] = q.z;
    } else {
        p[0] = a.x[i]; p[1] = a.y[i]; p[2] = a.z[i];
    }
    if (a.wrap) {
        float *dst[3] = {a.x_mut, a.y_mut, a.z_mut};
        for (int d = 0; d < 3; ++d)
            if (a.pbc[d] && isfinite(p[d])) {
                p[d] = wrap_coord(p[d], a.box[d]);
                if (!a.from_pos4) dst[d][i] = p[d];
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
    const int cid = cell_index(c[0], c[1], c[2], a.nc);
    a.cell_id[i] = cid;
    atomicAdd(&a.cell_count[cid], 1);
    a.pos4[i] = make_float4(p[0], p[1], p[2], (float)t);
    a.ref[i] = p[0];
    a.ref[a.n + i] = p[1];
    a.ref[2 * a.n + i] = p[2];
}

__global__ void k_nb_bin(NbArgs a) { nb_bin_body(a, blockIdx.x); }

// Exclusive scan, two phases.  Block b scans 1024 counts and leaves their
// total; a second pass adds to every count the totals of the blocks before
// its own (each workgroup sums those itself).
constexpr int SCAN_B = 1024;

__device__ __forceinline__ void scan_local_body(const NbArgs &a, int bx) {
    if (build_off(a)) return;
    const int32_t *in = a.cell_count;
    int32_t *out = a.cell_start, *block_sums = a.scan_tmp;
    const int n = a.ncell;
    __shared__ int32_t s[SCAN_B];
    int base = bx * SCAN_B;
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
    if (t == 0) block_sums[bx] = s[SCAN_B - 1];
}

__global__ void k_scan_local(NbArgs a) { scan_local_body(a, blockIdx.x); }

__device__ __forceinline__ void scan_add_body(const NbArgs &a, int bx) {
    if (build_off(a)) return;
    __shared__ int32_t off_s;
    const int nb = (a.ncell + SCAN_B - 1) / SCAN_B;
    const int sb = (bx * (int)blockDim.x) / SCAN_B;  // the scan block of this workgroup's cells
    if (threadIdx.x < 64) {
        // the totals of the blocks before it (integer sums: any order gives
        // the same), and in workgroup 0 the grand total after the last cell
        int32_t before = 0, all = 0;
        for (int b = threadIdx.x; b < nb; b += 64) {
            const int32_t v = a.scan_tmp[b];
            before += b < sb ? v : 0;
            all += v;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            before += __shfl_xor(before, o);
            all += __shfl_xor(all, o);
        }
        if (threadIdx.x == 0) {
            off_s = before;
            if (bx == 0) a.cell_start[a.ncell] = all;
        }
    }
    __syncthreads();
    const int k = bx * blockDim.x + threadIdx.x;
    if (k >= a.ncell) return;
    const int32_t v = a.cell_start[k] + off_s;
    a.cell_start[k] = v;
    a.cell_cursor[k] = v;
}

__global__ void k_scan_add(NbArgs a) { scan_add_body(a, blockIdx.x); }

__device__ __forceinline__ void nb_fill_body(const NbArgs &a, int bx) {
    if (build_off(a)) return;
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    int slot = atomicAdd(&a.cell_cursor[a.cell_id[i]], 1);
    a.cell_tmp[slot] = i;
}

__global__ void k_nb_fill(NbArgs a) { nb_fill_body(a, blockIdx.x); }

// rank of bead i among the members of its cell, by index
__device__ __forceinline__ void nb_rank_body(const NbArgs &a, int bx) {
    if (build_off(a)) return;
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int c = a.cell_id[i];
    const int s = a.cell_start[c], e = a.cell_start[c + 1];
    int rank = 0;
    for (int q = s; q < e; ++q) rank += (a.cell_tmp[q] < i) ? 1 : 0;
    a.cell_list[s + rank] = i;
    const float4 p = a.pos4[i];
    const uint32_t tag = (uint32_t)i | ((uint32_t)p.w << CODE_SHIFT);
    a.pos_sorted[s + rank] = make_float4(p.x, p.y, p.z, __uint_as_float(tag));
}

__global__ void k_nb_rank(NbArgs a) { nb_rank_body(a, blockIdx.x); }

// flags (or) and row maxima of the active lanes, one atomic per wave
__device__ __forceinline__ void wave_status(int32_t *status, int flags, int total, int na) {
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        flags |= __shfl_xor(flags, w);
        total = max(total, __shfl_xor(total, w));
        na = max(na, __shfl_xor(na, w));
    }
    const uint64_t act = __ballot(1);
    if (__lane_id() == __ffsll((unsigned long long)act) - 1) {
        if (flags) atomicOr(&status[0], flags);
        atomicMax(&status[1], total);
        atomicMax(&status[2], na);
    }
}

// wrapped cell index and periodic image of k = c0 + offset (|offset| <= 2,
// so at most two corrections); false for an open dimension outside the grid
__device__ __forceinline__ bool wrap_cell(int k, int nc, int pbc, int &kw, int &img) {
    img = 0;
    if (!pbc) {
        kw = k;
        return k >= 0 && k < nc;
    }
    while (k < 0) { k += nc; --img; }
    while (k >= nc) { k -= nc; ++img; }
    kw = k;
    return true;
}

// lower bound, in cell units, of the distance along one axis from a point at
// fractional position u in its cell to the cell at the given offset
__device__ __forceinline__ float cell_gap(int off, float u) {
    return off > 0 ? (float)off - u : (off < 0 ? (float)(-off - 1) + u : 0.0f);
}

// One of the four stacks of a row under construction.  Entries are kept in
// registers four at a time and written as one aligned 16-byte store (the rows
// of a wave lie far apart, so single 4-byte stores would each take a memory
// transaction); a stack that grows downwards stores its groups reversed.
// Groups that would leave the stack's region are dropped: the row then
// overflows and is discarded anyway.
struct RowStack {
    uint32_t b0, b1, b2, b3;  // the last four entries, oldest first
    int cnt;
    __device__ __forceinline__ void push(uint32_t e, uint32_t *row, int base, int limit, bool down) {
        b0 = b1;
        b1 = b2;
        b2 = b3;
        b3 = e;
        ++cnt;
        if ((cnt & 3) != 0 || cnt > limit) return;
        if (!down) *reinterpret_cast<uint4 *>(row + base + cnt - 4) = make_uint4(b0, b1, b2, b3);
        else *reinterpret_cast<uint4 *>(row + base - cnt + 1) = make_uint4(b3, b2, b1, b0);
    }
    // the entries of the last, incomplete group
    __device__ __forceinline__ void finish(uint32_t *row, int base, int limit, bool down) {
        const int r = cnt & 3;
        const uint32_t last[4] = {b0, b1, b2, b3};
#pragma unroll
        for (int q = 1; q <= 3; ++q) {
            if (q > r) break;
            const int k = cnt - q;  // insertion index of entry last[4 - q]
            if (k >= limit) continue;
            row[down ? base - k : base + k] = last[4 - q];
        }
    }
};

// the row of bead i; returns its flags, length and angular length
// thr[ti T + tj] = (list2R, list2A, in2A, in2R) of the type pair, in LDS
__device__ __forceinline__ void build_row(const NbArgs &a, const float4 *thr, const int i, int &flags_out,
                                          int &total_out, int &na_out) {
    const int n = a.n;
    const float4 pi = a.pos4[i];
    const int ti = (int)pi.w;
    const float4 *thr_i = thr + ti * a.T;
    int c0[3];
    float u[3];
    {
        const float pv[3] = {pi.x, pi.y, pi.z};
        for (int d = 0; d < 3; ++d) {
            const float f = mul_rn(pv[d], a.inv_cs[d]);
            c0[d] = cell_coord(pv[d], a.inv_cs[d], a.nc[d]);
            u[d] = fminf(fmaxf(f - (float)c0[d], 0.0f), 1.0f);
        }
    }
    const float cs[3] = {1.0f / a.inv_cs[0], 1.0f / a.inv_cs[1], 1.0f / a.inv_cs[2]};
    // four stacks in the row: angular inside r_c^A up from 0, angular shell
    // down from cap_A - 1, radial-only inside r_c^R up from cap_A, radial
    // shell down from cap_A + cap - 1.  Kept in this class order, the rows let
    // the lanes of a wave find their in-cutoff pairs in the same slots.
    const int A4 = (a.cap_A + 3) & ~3, R4 = (a.cap + 3) & ~3;
    uint32_t *row = a.rowbuf + (size_t)i * (A4 + R4);
    RowStack sai{0u, 0u, 0u, 0u, 0}, sas{0u, 0u, 0u, 0u, 0}, sri{0u, 0u, 0u, 0u, 0}, srs{0u, 0u, 0u, 0u, 0};
    int flags = 0;
    for (int dz = -a.m[2]; dz <= a.m[2]; ++dz) {
        int kz, iz;
        const bool vz = wrap_cell(c0[2] + dz, a.nc[2], a.pbc[2], kz, iz);
        const float gz = cell_gap(dz, u[2]) * cs[2];
        for (int dy = -a.m[1]; dy <= a.m[1]; ++dy) {
            int ky, iy;
            const bool vy = wrap_cell(c0[1] + dy, a.nc[1], a.pbc[1], ky, iy);
            const float gy = cell_gap(dy, u[1]) * cs[1];
            // the (up to five) cells of this row of offsets: indices and cull
            // tests first, then every candidate range is loaded before any
            // candidate is read, so the loads overlap instead of queueing
            const int wx = 2 * a.m[0] + 1;
            int cid5[5], ix5[5], s5[5], e5[5];
            bool use5[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                use5[k] = false;
                cid5[k] = 0;
                ix5[k] = 0;
                if (k < wx) {
                    const int dx = k - a.m[0];
                    int kx, ix;
                    const bool vx = wrap_cell(c0[0] + dx, a.nc[0], a.pbc[0], kx, ix);
                    const float gx = cell_gap(dx, u[0]) * cs[0];
                    // skip cells entirely beyond reach (a lower bound with margin)
                    use5[k] = vx && vy && vz && !(gx * gx + gy * gy + gz * gz > a.cull2);
                    cid5[k] = cell_index(kx, ky, kz, a.nc);
                    ix5[k] = ix;
                }
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                s5[k] = use5[k] ? a.cell_start[cid5[k]] : 0;
                e5[k] = use5[k] ? a.cell_start[cid5[k] + 1] : 0;
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                if (k >= wx) break;
                if (!use5[k]) continue;
                const int ix = ix5[k];
                const int s = s5[k], e = e5[k];
                if (ix < -2 || ix > 2 || iy < -2 || iy > 2 || iz < -2 || iz > 2) { flags |= NEP_FLAG_IMAGE_RANGE; continue; }
                // s = fl(n L), exact predicate with every operation rounded separately
                const float sx = mul_rn((float)ix, a.box[0]);
                const float sy = mul_rn((float)iy, a.box[1]);
                const float sz = mul_rn((float)iz, a.box[2]);
                const bool zero_shift = (ix == 0 && iy == 0 && iz == 0);
                const uint32_t code = (uint32_t)((ix + 2) + 5 * (iy + 2) + 25 * (iz + 2));
                for (int q0 = s; q0 < e; q0 += 4) {
                    // up to four independent loads in flight before any is used
                    float4 pb[4];
#pragma unroll
                    for (int u4 = 0; u4 < 4; ++u4) pb[u4] = a.pos_sorted[min(q0 + u4, e - 1)];
#pragma unroll
                    for (int u4 = 0; u4 < 4; ++u4) {
                    if (q0 + u4 >= e) break;
                    const float4 pj = pb[u4];
                    const uint32_t tag = __float_as_uint(pj.w);
                    const int j = (int)(tag & J_MASK);
                    // every component is used before any test, so the candidate
                    // arrives in one 16-byte load
                    const float ddx = sub_rn(add_rn(pj.x, sx), pi.x);
                    const float ddy = sub_rn(add_rn(pj.y, sy), pi.y);
                    const float ddz = sub_rn(add_rn(pj.z, sz), pi.z);
                    const float d2 = add_rn(add_rn(mul_rn(ddx, ddx), mul_rn(ddy, ddy)),
                                               mul_rn(ddz, ddz));
                    const float4 th = thr_i[tag >> CODE_SHIFT];
                    if (!(d2 < th.x) || (j == i && zero_shift)) continue;
                    if (d2 == 0.0f) flags |= NEP_FLAG_OVERLAP;
                    const uint32_t entry = (uint32_t)j | (code << CODE_SHIFT);
                    if (d2 < th.y) {
                        if (d2 < th.z) sai.push(entry, row, 0, A4, false);
                        else sas.push(entry, row, A4 - 1, A4, true);
                    } else {
                        if (d2 < th.w) sri.push(entry, row, A4, R4, false);
                        else srs.push(entry, row, A4 + R4 - 1, R4, true);
                    }
                    }
                }
            }
        }
    }
    sai.finish(row, 0, A4, false);
    sas.finish(row, A4 - 1, A4, true);
    sri.finish(row, A4, R4, false);
    srs.finish(row, A4 + R4 - 1, R4, true);
    const int nai = sai.cnt, nri = sri.cnt;
    const int na = nai + sas.cnt;
    const int total = na + nri + srs.cnt;
    if (na > a.cap_A) flags |= NEP_FLAG_OVERFLOW_A;
    if (total > a.cap) flags |= NEP_FLAG_OVERFLOW_R;
    const bool over = (flags & (NEP_FLAG_OVERFLOW_A | NEP_FLAG_OVERFLOW_R)) != 0;
    a.cnt[i] = over ? 0 : total;
    a.cnt[n + i] = over ? 0 : na;
    a.cls[i] = over ? 0 : (min(nai, 255) | (nri << 8));
    flags_out = flags;
    total_out = total;
    na_out = na;
}

__device__ __forceinline__ void nb_rows_body(const NbArgs &a, int bx, int gx) {
    if (build_off(a)) return;  // uniform over the grid
    __shared__ float4 thr[MAXT * MAXT];
    if (threadIdx.x < MAXT * MAXT) {
        const int k = threadIdx.x;
        thr[k] = make_float4(a.list2R[k], a.list2A[k], a.in2A[k], a.in2R[k]);
    }
    __syncthreads();
    const int i = xcd_tile(bx, gx) * BLOCK + threadIdx.x;
    int flags = 0, total = 0, na = 0;
    if (i < a.n) build_row(a, thr, i, flags, total, na);
    wave_status(a.status, flags, total, na);  // every lane takes part
}

__global__ __launch_bounds__(BLOCK) void k_nb_rows(NbArgs a) { nb_rows_body(a, blockIdx.x, gridDim.x); }

// row-major scratch -> slot-major lists: slot p of bead i is scratch entry p for
// the angular prefix, and the radial-only entries, kept from the back of the
// scratch row, follow in the order they were found.  A workgroup moves its
// 256 beads through LDS 16 slots at a time: each wave reads 16 consecutive
// slots of four rows, and writes one slot of 64 consecutive beads.
//
// The same workgroup writes the processing order of its beads for the fused
// kernel.  A bead's cost grows with its row (an angular pair inside r_c^A costs
// about twenty radial list entries), and a wave takes as long as its busiest
// lane, so the beads of the block (neighbours in space for a spatially ordered
// system) are ordered by decreasing cost, ties by index: the lanes of a wave
// then carry similar work.  The order only decides which thread evaluates
// which bead; every result is the same bit for bit.
constexpr int TR_SLOTS = 16;

__device__ __forceinline__ int row_src(int p, int na, int nai, int nri, int A4, int R4) {
    if (p < nai) return p;                            // inside r_c^A
    if (p < na) return A4 - 1 - (p - nai);            // angular shell
    if (p < na + nri) return A4 + (p - na);           // inside r_c^R
    return A4 + R4 - 1 - (p - na - nri);              // radial shell
}

__device__ __forceinline__ void nb_transpose_body(const NbArgs &a, int bx, int gx) {
    if (build_off(a)) return;  // uniform over the grid
    __shared__ uint32_t tile[TR_SLOTS][BLOCK + 4];
    __shared__ int4 info[BLOCK];  // total, angular, inside r_c^A, inside r_c^R (radial-only)
    __shared__ int4 cost4[BLOCK / 4];  // processing cost of each bead (-1 past the system's end)
    __shared__ int max_total;
    const int n = a.n;
    const int i0 = xcd_tile(bx, gx) * BLOCK;
    const int A4 = (a.cap_A + 3) & ~3, R4 = (a.cap + 3) & ~3;
    int4 f = make_int4(0, 0, 0, 0);
    if (i0 + (int)threadIdx.x < n) {
        const int i = i0 + threadIdx.x;
        const int c = a.cls[i];
        f = make_int4(a.cnt[i], a.cnt[n + i], c & 255, c >> 8);
    }
    info[threadIdx.x] = f;
    reinterpret_cast<int *>(cost4)[threadIdx.x] = i0 + (int)threadIdx.x < n ? 20 * f.z + f.x : -1;
    if (threadIdx.x == 0) max_total = 0;
    __syncthreads();
    int m = f.x;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) m = max(m, __shfl_xor(m, w));
    if (__lane_id() == 0) atomicMax(&max_total, m);
    __syncthreads();
    const int mt = max_total;
    if (a.order) {
        // rank of this bead among the block's beads by decreasing cost (ties
        // by index; the -1 of missing beads ranks below every cost), four
        // costs per LDS read
        const int b = threadIdx.x;
        const int nb = min(BLOCK, n - i0);
        const int cost = 20 * f.z + f.x;
        int rank = 0;
#pragma unroll 4
        for (int k4 = 0; k4 < BLOCK / 4; ++k4) {
            const int4 c = cost4[k4];
            const int cs[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 4 * k4 + u;
                rank += (cs[u] > cost || (cs[u] == cost && k < b)) ? 1 : 0;
            }
        }
        if (b < nb) a.order[i0 + rank] = i0 + b;
    }
    constexpr int BEADS_PER_PASS = BLOCK / TR_SLOTS;
    const int pl = threadIdx.x % TR_SLOTS, bsub = threadIdx.x / TR_SLOTS;
    for (int p0 = 0; p0 < mt; p0 += TR_SLOTS) {
        // all TR_SLOTS loads are issued before any is used: unconditional, at a
        // slot clamped into the row (and a bead clamped into the system), so
        // none waits behind a branch; slots past a row's end are never read
        uint32_t vals[TR_SLOTS];
#pragma unroll
        for (int k = 0; k < TR_SLOTS; ++k) {
            const int b = bsub + k * BEADS_PER_PASS;
            const int4 g = info[b];
            const int p = min(p0 + pl, max(g.x - 1, 0));
            const int bead = min(i0 + b, n - 1);
            vals[k] = a.rowbuf[(size_t)bead * (A4 + R4) + row_src(p, g.y, g.z, g.w, A4, R4)];
        }
#pragma unroll
        for (int k = 0; k < TR_SLOTS; ++k) tile[pl][bsub + k * BEADS_PER_PASS] = vals[k];
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < TR_SLOTS; ++q)
            if (p0 + q < f.x) a.nbr[(size_t)(p0 + q) * n + i0 + threadIdx.x] = tile[q][threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_nb_transpose(NbArgs a) { nb_transpose_body(a, blockIdx.x, gridDim.x); }

// angular slots per thread: p = blockIdx.y + k gridDim.y (with the searches
// ending early, two per thread measured faster than one, three or four)
constexpr int REV_SLOTS = 2;

// Reverse entries of up to REV_SLOTS angular slots of bead i (slots by,
// by + gy, ...): where each neighbour j's row holds i with the opposite
// image.  The search scans j's angular entries in the row-major build rows,
// where they lie together (the entries inside r_c^A from the front, the
// angular shell entries from the end of the angular part), 16 bytes at a
// time; the searches of one thread advance together so their loads overlap.
// Lanes of a wave handle consecutive beads at the same slots.
__device__ __forceinline__ void nb_reverse_body(const NbArgs &a, int bx, int gx, int by, int gy) {
    if (build_off(a)) return;
    const int n = a.n;
    const int i = xcd_tile(bx, gx) * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int na = a.cnt[n + i];
    const int A4 = (a.cap_A + 3) & ~3, R4 = (a.cap + 3) & ~3;
    int p[REV_SLOTS], j[REV_SLOTS], nin[REV_SLOTS], lo[REV_SLOTS], nch[REV_SLOTS], found[REV_SLOTS];
    int ca[REV_SLOTS], cs[REV_SLOTS];
    bool sfirst[REV_SLOTS];
    uint32_t want[REV_SLOTS];
    // this bead's own class split: slots [0, nai_i) inside r_c^A, the rest in the shell
    const int nai_i = min(a.cls[i] & 255, na);
#pragma unroll
    for (int k = 0; k < REV_SLOTS; ++k) {
        p[k] = by + k * gy;
        const uint32_t e = p[k] < na ? a.nbr[(size_t)p[k] * n + i] : 0u;
        j[k] = (int)(e & J_MASK);
        want[k] = (uint32_t)i | ((124u - (e >> CODE_SHIFT)) << CODE_SHIFT);
        found[k] = -1;
        // a pair has the same class in both rows except where rounding puts its
        // distance on the two sides of r_c^A: search j's part of that class
        // first, then the other part
        sfirst[k] = p[k] >= nai_i;
    }
#pragma unroll
    for (int k = 0; k < REV_SLOTS; ++k) {
        const bool v = p[k] < na;
        // j's angular entries (0 after an overflow of j's row): nin inside
        // r_c^A at row positions [0, nin), the shell at [lo, A4)
        const int naj = v ? a.cnt[n + j[k]] : 0;
        const int nai = v ? min(a.cls[j[k]] & 255, naj) : 0;
        nin[k] = nai;
        lo[k] = A4 - (naj - nai);
        ca[k] = (nai + 3) >> 2;                                         // chunks inside r_c^A
        cs[k] = naj > nai ? (A4 - (lo[k] & ~3)) >> 2 : 0;               // chunks of the shell
        nch[k] = ca[k] + cs[k];
    }
    int most = 0;
#pragma unroll
    for (int k = 0; k < REV_SLOTS; ++k) most = max(most, nch[k]);
    for (int c = 0; c < most; ++c) {
        bool done = true;
#pragma unroll
        for (int k = 0; k < REV_SLOTS; ++k) done = done && (c >= nch[k] || found[k] >= 0);
        if (done) break;
#pragma unroll
        for (int k = 0; k < REV_SLOTS; ++k) {
            if (c >= nch[k] || found[k] >= 0) continue;
            const bool shell = sfirst[k] ? c < cs[k] : c >= ca[k];
            const int cc = sfirst[k] ? (shell ? c : c - cs[k]) : (shell ? c - ca[k] : c);
            const int q0 = shell ? (lo[k] & ~3) + 4 * cc : 4 * cc;
            const uint4 w = *reinterpret_cast<const uint4 *>(a.rowbuf + (size_t)j[k] * (A4 + R4) + q0);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u;
                const bool in_range = shell ? (q >= lo[k] && q < A4) : (q < nin[k]);
                // slot of row position q: itself inside r_c^A, counted from the
                // end of the angular part in the shell
                if (found[k] < 0 && in_range && ws[u] == want[k]) found[k] = shell ? nin[k] + (A4 - 1 - q) : q;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < REV_SLOTS; ++k)
        if (p[k] < na) a.rev[(size_t)p[k] * n + i] = found[k] < 0 ? -1 : (int32_t)((size_t)found[k] * n + j[k]);
}

__global__ __launch_bounds__(BLOCK) void k_nb_reverse(NbArgs a) {
    nb_reverse_body(a, blockIdx.x, gridDim.x, blockIdx.y, gridDim.y);
}



hipError_t launch_build(const NbArgs &a, hipStream_t s) {
    int nbk = (a.n + BLOCK - 1) / BLOCK;
    int cbk = (a.ncell + BLOCK - 1) / BLOCK;
    if (!a.skip_clear)
        hipLaunchKernelGGL(k_nb_clear, dim3(cbk > 0 ? (cbk < 4096 ? cbk : 4096) : 1), dim3(BLOCK), 0, s,
                           a.ncell, a.cell_count, a.status, a.clear_status, a.ctrl);
    if (a.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_nb_bin, dim3(nbk), dim3(BLOCK), 0, s, a);
    int sb = (a.ncell + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_local, dim3(sb), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_scan_add, dim3(cbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_fill, dim3(nbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_rank, dim3(nbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_rows, dim3(nbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_transpose, dim3(nbk), dim3(BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_nb_reverse, dim3(nbk, (a.cap_A + REV_SLOTS - 1) / REV_SLOTS), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}



// ---- one launch per phase over the builds of many systems ----
// start[ph][r] is the first block of system r in phase ph (tables of
// n_sys + 1 entries, one per tile kind: cells to clear, beads, scan blocks,
// cells to offset, and (bead, slot-group) pairs).
enum { NB_TILE_CLEAR = 0, NB_TILE_BEAD, NB_TILE_SCANL, NB_TILE_SCANA, NB_TILE_REV, NB_TILES };
static_assert(NB_TILES == NB_BATCH_TILES, "tile kinds of the batched build");
enum { OP_CLEAR, OP_BIN, OP_SCANL, OP_SCANA, OP_FILL, OP_RANK, OP_ROWS, OP_TRANSPOSE, OP_REVERSE };

template <int OP>
__global__ __launch_bounds__(BLOCK) void k_nb_batch(NbBatchArgs b) {
    constexpr int TILE = OP == OP_CLEAR ? NB_TILE_CLEAR
                         : OP == OP_SCANL ? NB_TILE_SCANL
                         : OP == OP_SCANA ? NB_TILE_SCANA
                         : OP == OP_REVERSE ? NB_TILE_REV
                                            : NB_TILE_BEAD;
    const int *st = b.start + TILE * (b.n_sys + 1);
    int lo = 0, hi = b.n_sys - 1;  // last system whose first block is <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const NbArgs &a = b.args[lo];
    const int bx = blockIdx.x - st[lo], gx = st[lo + 1] - st[lo];
    if constexpr (OP == OP_CLEAR) nb_clear_body(a.ncell, a.cell_count, a.status, a.clear_status, a.ctrl, bx, gx);
    if constexpr (OP == OP_BIN) nb_bin_body(a, bx);
    if constexpr (OP == OP_SCANL) scan_local_body(a, bx);
    if constexpr (OP == OP_SCANA) scan_add_body(a, bx);
    if constexpr (OP == OP_FILL) nb_fill_body(a, bx);
    if constexpr (OP == OP_RANK) nb_rank_body(a, bx);
    if constexpr (OP == OP_ROWS) nb_rows_body(a, bx, gx);
    if constexpr (OP == OP_TRANSPOSE) nb_transpose_body(a, bx, gx);
    if constexpr (OP == OP_REVERSE) {
        const int nbk = (a.n + BLOCK - 1) / BLOCK;
        nb_reverse_body(a, bx % nbk, nbk, bx / nbk, gx / nbk);
    }
}

void nb_batch_tiles(const NbArgs &a, int counts[NB_BATCH_TILES]) {
    const int nbk = (a.n + BLOCK - 1) / BLOCK;
    const int cbk = (a.ncell + BLOCK - 1) / BLOCK;
    counts[NB_TILE_CLEAR] = cbk > 0 ? (cbk < 4096 ? cbk : 4096) : 1;
    counts[NB_TILE_BEAD] = nbk;
    counts[NB_TILE_SCANL] = (a.ncell + SCAN_B - 1) / SCAN_B;
    counts[NB_TILE_SCANA] = cbk;
    counts[NB_TILE_REV] = nbk * ((a.cap_A + REV_SLOTS - 1) / REV_SLOTS);
}

hipError_t launch_build_batch(const NbBatchArgs &b, const int totals[NB_BATCH_TILES], hipStream_t s) {
    if (b.n_sys == 0) return hipSuccess;
#define NB_LAUNCH(OPC, TILEK)                                                                     \
    if (totals[TILEK] > 0) hipLaunchKernelGGL(k_nb_batch<OPC>, dim3(totals[TILEK]), dim3(BLOCK), 0, s, b);
    NB_LAUNCH(OP_CLEAR, NB_TILE_CLEAR)
    NB_LAUNCH(OP_BIN, NB_TILE_BEAD)
    NB_LAUNCH(OP_SCANL, NB_TILE_SCANL)
    NB_LAUNCH(OP_SCANA, NB_TILE_SCANA)
    NB_LAUNCH(OP_FILL, NB_TILE_BEAD)
    NB_LAUNCH(OP_RANK, NB_TILE_BEAD)
    NB_LAUNCH(OP_ROWS, NB_TILE_BEAD)
    NB_LAUNCH(OP_TRANSPOSE, NB_TILE_BEAD)
    NB_LAUNCH(OP_REVERSE, NB_TILE_REV)
#undef NB_LAUNCH
    return hipGetLastError();
}

}  // namespace nep
