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
//   4. rows:    one wavefront per cell stages the candidates of the cell's
//               (2m+1)^3 neighbour cells in registers, in a fixed order
//               (offset in (dz, dy, dx) order, then cell order), and tests the
//               cell's beads against them with the lanes over the candidates
//               (the exact float32 predicate); each row is assembled in LDS by
//               class (angular inside r_c^A, angular shell, radial-only
//               inside r_c^R, radial shell) and written slot-major into the
//               list, with its angular part's sort keys row-major
//   5. order:   the fused kernel's processing order, from the row lengths
//               (one launch with step 6)
//   6. reverse: for every angular entry, the mirrored entry is looked up by
//               its sort key among the neighbour's angular keys
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

// A build inside an MD run is skipped unless the drift's rebuild test, the
// pair test or the schedule asked for one (ctrl[0] == 1), and once the run is
// frozen after a failed build.  The test is uniform over the grid.
__device__ __forceinline__ bool build_off(const int32_t *ctrl, const int32_t *status, int clear_status) {
    if (ctrl && ctrl[0] != 1) return true;
    return !clear_status && (status[0] & FREEZE_MASK);
}
// Gate 2: the pair test decides (its verdict in fast[3]).
__device__ __forceinline__ bool build_off(const NbArgs &a) {
    if (a.ctrl && a.ctrl[0] == 2) {
        if (!(a.fast && a.fast[3])) return true;
        return !a.clear_status && (a.status[0] & FREEZE_MASK);
    }
    return build_off(a.ctrl, a.status, a.clear_status);
}

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
// it belongs to the lists, which the call continues from; the pair test's
// words cleared (its cell data must come from a build of this call)
__global__ void k_md_clear(int32_t *status, int32_t *ctrl, int gate0, int32_t *fast) {
    int t = threadIdx.x;
    if (t < 3) status[t] = 0;
    if (ctrl && t < 4) ctrl[t] = t == 0 ? gate0 : (t == 3 ? -1 : 0);  // [3]: no list built by this call yet
    if (fast && t < 4) fast[t] = 0;
}

hipError_t launch_clear_status(int32_t *status, int32_t *ctrl, int gate0, hipStream_t s, int32_t *fast) {
    hipLaunchKernelGGL(k_md_clear, dim3(1), dim3(64), 0, s, status, ctrl, gate0, fast);
    return hipGetLastError();
}

__device__ __forceinline__ int cell_coord(float x, float inv_cs, int nc) {
    float f = floorf(mul_rn(x, inv_cs));
    int k = (int)fminf(fmaxf(f, -1.0f), (float)nc);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

// grid coordinates of cell c: the inverse of cell_index
__device__ __forceinline__ void cell_coords(int c, const int nc[3], int xyz[3]) {
    constexpr int B = CELL_TILE;
    const int slab = B * nc[1] * nc[0];
    const int tz = c / slab;
    int r = c - tz * slab;
    const int hz = min(B, nc[2] - tz * B);
    const int trow = B * nc[0] * hz;
    const int ty = r / trow;
    r -= ty * trow;
    const int hy = min(B, nc[1] - ty * B);
    const int tile = B * hy * hz;
    const int tx = r / tile;
    r -= tx * tile;
    const int hx = min(B, nc[0] - tx * B);
    const int yz = r / hx;
    xyz[0] = tx * B + (r - yz * hx);
    xyz[1] = ty * B + yz % hy;
    xyz[2] = tz * B + yz / hy;
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
    if (bx == 0 && threadIdx.x == 0) {
        if (a.skip_clear && a.ctrl) a.ctrl[1] += 1;  // the clear phase's count
        if (a.fast) {
            a.fast[2] = 1;  // the pair test may use this build's cells
            a.ctrl[3] = 0;  // the new lists have served no step yet
        }
    }
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
    // the cell's coordinates, for the row kernel (one thread per cell here,
    // where the row kernel would compute them in every lane of a wave)
    int xyz[3];
    cell_coords(k, a.nc, xyz);
    a.cell_xyz[k] = xyz[0] | (xyz[1] << 10) | (xyz[2] << 20);
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
        // every wave of a build updates the same three words: an update that
        // cannot change a word is skipped (a stale read only costs an atomic)
        if (flags) atomicOr(&status[0], flags);
        if (total > __hip_atomic_load(&status[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&status[1], total);
        if (na > __hip_atomic_load(&status[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&status[2], na);
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

// ---- 4. rows ----
// One wavefront per home cell.  It loads the candidates of the cell's
// (2m+1)^3 neighbour cells once, into registers (candidate t = 64 k + lane in
// lane `lane`, batch k), in the fixed order of the search (offset in
// (dz, dy, dx) order, then cell order), each shifted by the periodic image of
// its offset and tagged with its list entry and its sort key; then it tests
// every bead of the cell against them, the lanes over the candidates.  A home
// bead's entries are appended in LDS in search order with their class (one
// ballot per 64 candidates and each lane's count of the set bits below it),
// and written out by class (angular inside r_c^A, angular shell, radial-only
// inside r_c^R, radial shell; search order within a class): slot-major into
// the list, and the angular keys row-major for the reverse search.  A row is
// thus the same, entry for entry, as a walk over the cells in that order.
//
// The key of an entry is its neighbour-cell offset index o (0..W-1 in search
// order) << 25 | the neighbour's position in cell order; within each class
// the keys of a row ascend (the reverse search reads a part linearly).  Bead i sits in the row of its neighbour j at the
// mirrored offset W-1-o, so the key it has there is known before j's row is
// read: the row kernel leaves that key in rev, and the reverse kernel finds
// its position in j's row.
constexpr int ROW_BATCHES = 8;                // candidates per lane held at a time
constexpr int ROW_WIN = 64 * ROW_BATCHES;     // candidates held by the wave
constexpr int ROW_OFF = 128;                  // room for the (2m+1)^3 <= 125 offsets
constexpr int ROW_HOME = 64;                  // home beads whose positions are staged in LDS
constexpr uint32_t ZERO_CODE = 62;            // image code of the zero shift, (0+2) + 5 (0+2) + 25 (0+2)

struct RowsLds {
    float4 thr[MAXT * MAXT];  // (list2R, list2A, in2A, in2R) of the type pair
    float4 home[ROW_HOME];    // positions and tags of the cell's first beads
    int beg[ROW_OFF];         // first cell-order index of the offset's cell
    int pre[ROW_OFF];         // first flat candidate index of the offset
    float sh[3][ROW_OFF];     // periodic shift of the offset
    uint32_t code[ROW_OFF];   // image code of the offset, in entry position
    uint8_t owner[ROW_WIN];   // offset of each candidate of the window
};

// bytes of dynamic LDS of the row kernel: the entries and keys of the row
// under construction, in the order found (A4 + R4 of them, then a trash slot
// per lane), and their classes
__host__ __device__ __forceinline__ int row_lds_bytes(int cap, int cap_A) {
    const int w = ((cap_A + 3) & ~3) + ((cap + 3) & ~3) + 64;
    return (w * 8 + w + 15) & ~15;  // a multiple of 16 bytes
}

// The row kernel's workgroup is a single wavefront, whose LDS operations
// complete in issue order: a compiler barrier with wavefront-scope fences is
// all that orders one lane's LDS writes before another lane's reads (a
// workgroup barrier would also wait for every global store in flight).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// number of set bits of m below this lane
__device__ __forceinline__ int bits_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// candidates of one window, one batch of 64 per register slot
struct Cands {
    float x[ROW_BATCHES], y[ROW_BATCHES], z[ROW_BATCHES];
    uint32_t ent[ROW_BATCHES];  // j | image code << 25
    uint32_t key[ROW_BATCHES];  // offset << 25 | cell-order index
    uint32_t types;             // 2 bits per batch
};

// Candidates [base, base + ROW_WIN) of the flat sequence into registers.
// Lane `lane` owns offsets o = lane + 64 hf (hf = 0, 1) with cnt2[hf]
// candidates from flat index pre2[hf].  With home_from >= 0 the lanes also
// stage the positions of the cell's first beads (cell-order index home_from
// on) in LDS.
__device__ __forceinline__ void stage_window(const NbArgs &a, RowsLds &L, int base, int total, const int cnt2[2],
                                             const int pre2[2], int home_from, int nh, Cands &C) {
    const int lane = threadIdx.x;
    wave_sync();  // the previous window's owners are no longer read
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        const int lo = max(pre2[hf], base), hi = min(pre2[hf] + cnt2[hf], base + ROW_WIN);
        for (int t = lo; t < hi; ++t) L.owner[t - base] = (uint8_t)(lane + 64 * hf);
    }
    wave_sync();
    const int nw = min(ROW_WIN, total - base);
#pragma unroll
    for (int k = 0; k < ROW_BATCHES; ++k) {
        const int t = 64 * k + lane;
        const int o = t < nw ? L.owner[t] : 0;
        const int q = t < nw ? L.beg[o] + (base + t - L.pre[o]) : 0;
        C.key[k] = ((uint32_t)o << CODE_SHIFT) | (uint32_t)q;
    }
    // every load issued before any is used (lanes past the window read bead 0)
    const bool hl = home_from >= 0 && lane < min(nh, ROW_HOME);
    const float4 hp = hl ? a.pos_sorted[home_from + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < ROW_BATCHES; ++k) {
        const float4 p = a.pos_sorted[C.key[k] & J_MASK];
        C.x[k] = p.x;
        C.y[k] = p.y;
        C.z[k] = p.z;
        C.ent[k] = __float_as_uint(p.w);
    }
    if (hl) L.home[lane] = hp;
    C.types = 0;
#pragma unroll
    for (int k = 0; k < ROW_BATCHES; ++k) {
        const int o = (int)(C.key[k] >> CODE_SHIFT);
        const uint32_t tag = C.ent[k];
        // a lane past the window gets a candidate at infinity: its squared
        // distance is +inf, below no cutoff
        if (64 * k + lane >= nw) C.x[k] = INFINITY;
        C.x[k] = add_rn(C.x[k], L.sh[0][o]);
        C.y[k] = add_rn(C.y[k], L.sh[1][o]);
        C.z[k] = add_rn(C.z[k], L.sh[2][o]);
        C.ent[k] = (tag & J_MASK) | L.code[o];
        C.types |= (tag >> CODE_SHIFT) << (2 * k);
    }
    wave_sync();
}

// the rows of the beads of cell c; one wavefront, all lanes.  MT: more than
// one bead type (per-lane thresholds)
template <bool MT>
__device__ __forceinline__ void row_cell(const NbArgs &a, int c, RowsLds &L, uint32_t *row, int &flags, int &most,
                                         int &most_a) {
    const int lane = threadIdx.x;
    const int n = a.n;
    const int A4 = (a.cap_A + 3) & ~3, R4 = (a.cap + 3) & ~3;
    const int cap4 = A4 + R4;           // entries held for a row
    const int trash = cap4;             // trash slots [cap4, cap4 + 64)
    uint2 *rows = reinterpret_cast<uint2 *>(row);           // (entry, key) in the order found
    uint8_t *rcls = reinterpret_cast<uint8_t *>(rows + cap4 + 64);  // their classes
    const int w0 = 2 * a.m[0] + 1, w1 = 2 * a.m[1] + 1;
    const int W = w0 * w1 * (2 * a.m[2] + 1);
    const int o_home = (W - 1) / 2;  // the zero offset (always in the first half)
    const int32_t xyz = a.cell_xyz[c];
    const int c0[3] = {xyz & 1023, (xyz >> 10) & 1023, xyz >> 20};
    wave_sync();  // the previous cell's tables are no longer read
    // offsets o = lane and lane + 64: cell range, shift, image code, and the
    // exclusive prefix of the candidate counts
    int cnt2[2], beg2[2], pre2[2], total = 0;
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        const int o = lane + 64 * hf;
        int cid = -1;
        if (o < W) {
            // o = (oz w1 + oy) w0 + ox; o < 128, so the float quotients are exact
            const int qx = (int)(((float)o + 0.5f) * (1.0f / (float)w0));
            const int qy = (int)(((float)qx + 0.5f) * (1.0f / (float)w1));
            const int off[3] = {o - qx * w0 - a.m[0], qx - qy * w1 - a.m[1], qy - a.m[2]};
            int k[3], img[3];
            bool ok = true;
            float g2 = 0.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ok = wrap_cell(c0[d] + off[d], a.nc[d], a.pbc[d], k[d], img[d]) && ok;
                // gap between the two cells along d: a lower bound for every
                // bead of the home cell (the cull has the build's margin)
                const float g = (float)max(abs(off[d]) - 1, 0) * (1.0f / a.inv_cs[d]);
                g2 = add_rn(g2, mul_rn(g, g));
            }
            ok = ok && !(g2 > a.cull2);
            if (ok && (img[0] < -2 || img[0] > 2 || img[1] < -2 || img[1] > 2 || img[2] < -2 || img[2] > 2)) {
                flags |= NEP_FLAG_IMAGE_RANGE;
                ok = false;
            }
            if (ok) {
                cid = cell_index(k[0], k[1], k[2], a.nc);
#pragma unroll
                for (int d = 0; d < 3; ++d) L.sh[d][o] = mul_rn((float)img[d], a.box[d]);
                L.code[o] = (uint32_t)((img[0] + 2) + 5 * (img[1] + 2) + 25 * (img[2] + 2)) << CODE_SHIFT;
            }
        }
        beg2[hf] = cid >= 0 ? a.cell_start[cid] : 0;
        cnt2[hf] = cid >= 0 ? a.cell_start[cid + 1] : 0;
    }
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        const int o = lane + 64 * hf;
        cnt2[hf] -= beg2[hf];
        const int incl = wave_incl_scan(cnt2[hf]);
        pre2[hf] = total + incl - cnt2[hf];
        if (o < W) {
            L.beg[o] = beg2[hf];
            L.pre[o] = pre2[hf];
        }
        total += __builtin_amdgcn_readfirstlane(__shfl(incl, 63));
    }
    // (values the same in every lane, held in scalar registers so that the
    // loops below are uniform)
    const int s_c = __builtin_amdgcn_readfirstlane(__shfl(beg2[0], o_home));
    const int nh = __builtin_amdgcn_readfirstlane(__shfl(cnt2[0], o_home));
    if (nh <= 0) return;
    Cands C;
    const bool one = total <= ROW_WIN;  // one window: staged once for all home beads
    for (int h = 0; h < nh; ++h) {
        const int qh = s_c + h;
        // window 0 in registers (and, for the first bead, the home positions in LDS)
        if (h == 0 || !one) stage_window(a, L, 0, total, cnt2, pre2, h == 0 ? s_c : -1, nh, C);
        // the home bead and its type's thresholds against each candidate type
        // (the same in every lane)
        const float4 ph = h < ROW_HOME ? L.home[h] : a.pos_sorted[qh];
        const uint32_t tagh = __float_as_uint(ph.w);
        const int ih = (int)(tagh & J_MASK);
        const int tb = (int)(tagh >> CODE_SHIFT) * a.T;
        const float4 th0 = L.thr[tb];
        const float4 th1 = MT ? L.thr[tb + min(1, a.T - 1)] : th0;
        const float4 th2 = MT ? L.thr[tb + min(2, a.T - 1)] : th0;
        const float4 th3 = MT ? L.thr[tb + min(3, a.T - 1)] : th0;
        const uint32_t self = (uint32_t)ih | (ZERO_CODE << CODE_SHIFT);
        // every entry inside the list cutoff in the order found (one ballot
        // per batch), with its class: 0 angular inside r_c^A, 1 angular shell,
        // 2 radial-only inside r_c^R, 3 radial shell; the class counts from
        // the same ballots
        int cnt = 0, n0 = 0, n1 = 0, n2 = 0;
        uint64_t overlap = 0;
        for (int base = 0; base < total; base += ROW_WIN) {
            if (base > 0) stage_window(a, L, base, total, cnt2, pre2, -1, nh, C);
            const int nw = min(ROW_WIN, total - base);
#pragma unroll
            for (int k = 0; k < ROW_BATCHES; ++k) {
                if (64 * k >= nw) break;
                const uint32_t tj = MT ? (C.types >> (2 * k)) & 3u : 0u;
                const float4 th = tj == 0 ? th0 : (tj == 1 ? th1 : (tj == 2 ? th2 : th3));
                // the exact predicate, every operation rounded on its own
                const float ddx = sub_rn(C.x[k], ph.x);
                const float ddy = sub_rn(C.y[k], ph.y);
                const float ddz = sub_rn(C.z[k], ph.z);
                const float d2 = add_rn(add_rn(mul_rn(ddx, ddx), mul_rn(ddy, ddy)), mul_rn(ddz, ddz));
                const uint32_t ent = C.ent[k];
                const uint64_t m_in = __ballot(d2 < th.x) & ~__ballot(ent == self);
                const uint64_t m_a = __ballot(d2 < th.y), m_ai = __ballot(d2 < th.z), m_ri = __ballot(d2 < th.w);
                overlap |= m_in & __ballot(d2 == 0.0f);
                const bool in = d2 < th.x && ent != self;
                const uint32_t cl = d2 < th.y ? (d2 < th.z ? 0u : 1u) : (d2 < th.w ? 2u : 3u);
                const int pos = cnt + bits_below(m_in);
                const int w = in && pos < cap4 ? pos : trash + lane;
                rows[w] = make_uint2(ent, C.key[k]);
                rcls[w] = (uint8_t)cl;
                cnt += (int)__popcll(m_in);
                n0 += (int)__popcll(m_in & m_a & m_ai);
                n1 += (int)__popcll(m_in & m_a & ~m_ai);
                n2 += (int)__popcll(m_in & ~m_a & m_ri);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (overlap) flags |= NEP_FLAG_OVERLAP;
        const int nf = min(cnt, cap4);
        const int nai = n0, na = n0 + n1, nri = n2, tot = cnt;
        int fl = 0;
        if (na > a.cap_A) fl |= NEP_FLAG_OVERFLOW_A;
        if (tot > a.cap) fl |= NEP_FLAG_OVERFLOW_R;
        flags |= fl;
        most = max(most, tot);
        most_a = max(most_a, na);
        const bool over = fl != 0;
        uint32_t *ar = a.arow + (size_t)ih * (4 + A4);
        if (lane == 0) {
            a.cnt[ih] = over ? 0 : tot;
            a.cnt[n + ih] = over ? 0 : na;
            a.cls[ih] = over ? 0 : (min(nai, 255) | (nri << 8));
            *reinterpret_cast<uint4 *>(ar) = make_uint4(over ? 0u : (uint32_t)nai, over ? 0u : (uint32_t)na, 0u, 0u);
        }
        wave_sync();  // the row is complete
        if (!over) {
            // the entries in class order (found order within a class), 64 at a
            // time: each lane's slot from its class's ballot, then one store
            // of each kind for the lanes together
            int run[4] = {0, nai, na, na + nri};  // next slot of each class
            for (int u0 = 0; u0 < nf; u0 += 64) {
                const bool v = u0 + lane < nf;
                const int cl = v ? rcls[u0 + lane] : 4;
                const uint2 e = rows[v ? u0 + lane : 0];
                uint64_t mine = 0;
                int start = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t m = __ballot(cl == q);
                    mine = cl == q ? m : mine;
                    start = cl == q ? run[q] : start;
                    run[q] += (int)__popcll(m);
                }
                const int r = start + bits_below(mine);  // slot
                if (v) {
                    a.nbr[(size_t)r * n + ih] = e.x;
                    if (cl < 2) {
                        // angular keys: inside r_c^A up from word 4, the shell
                        // down from the row's end; the key this bead has in the
                        // neighbour's row waits in rev
                        ar[cl == 0 ? 4 + r : 4 + A4 - 1 - (r - nai)] = e.y;
                        a.rev[(size_t)r * n + ih] =
                            (int32_t)((((uint32_t)(W - 1) - (e.y >> CODE_SHIFT)) << CODE_SHIFT) | (uint32_t)qh);
                    }
                }
            }
        }
        wave_sync();  // the row is free for the next bead
    }
}

__device__ __forceinline__ void rows_thresholds(const NbArgs &a, RowsLds &L) {
    const int k = threadIdx.x;
    if (k < MAXT * MAXT) L.thr[k] = make_float4(a.list2R[k], a.list2A[k], a.in2A[k], a.in2R[k]);
}

// One workgroup (a single wavefront) per cell, consecutive cells on one XCD;
// the hardware dispatcher balances the cells' uneven work as it goes.
// Measured on the 216,000-bead lists (a rebuild / a launch that finds no
// rebuild due): a cell per workgroup 0.24 ms / 15.5 us; two, four or eight
// single-cell waves per workgroup 0.27 / 0.32 / 0.34 ms and 8.3 / 4.9 / 4.9 us
// (a workgroup's LDS is held until its busiest cell is done); two, four or
// eight consecutive cells per wavefront 0.30-0.44 ms; a persistent grid taking
// cells from per-XCD counters 0.85 ms / 4.6 us (device-scope atomics from all
// XCDs on one line serialise).
template <bool MT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_nb_rows(NbArgs a) {
    extern __shared__ __align__(16) uint32_t row_dyn[];
    __shared__ RowsLds L;
    if (build_off(a)) return;  // uniform over the grid
    rows_thresholds(a, L);
    int flags = 0, most = 0, most_a = 0;
    row_cell<MT>(a, xcd_tile(blockIdx.x, gridDim.x), L, row_dyn, flags, most, most_a);
    wave_status(a.status, flags, most, most_a);
}

// Processing order of the fused kernel.  A bead's cost grows with its row (an
// angular pair inside r_c^A costs about twenty radial list entries), and a
// wave takes as long as its busiest lane, so the beads of each block of 256
// (neighbours in space for a spatially ordered system) are ordered by
// decreasing cost, ties by index: the lanes of a wave then carry similar
// work.  The order only decides which thread evaluates which bead; every
// result is the same bit for bit.
__device__ __forceinline__ void nb_order_body(const NbArgs &a, int bx, int gx) {
    if (build_off(a) || !a.order) return;  // uniform over the grid
    __shared__ int4 cost4[BLOCK / 4];
    const int n = a.n;
    const int i0 = xcd_tile(bx, gx) * BLOCK;
    const int b = threadIdx.x;
    int cost = -1;  // below every cost: past the system's end
    if (i0 + b < n) cost = 20 * (a.cls[i0 + b] & 255) + a.cnt[i0 + b];
    reinterpret_cast<int *>(cost4)[b] = cost;
    __syncthreads();
    const int nb = min(BLOCK, n - i0);
    int rank = 0;
#pragma unroll 4
    for (int k4 = 0; k4 < BLOCK / 4; ++k4) {
        const int4 c = cost4[k4];
        const int cv[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = 4 * k4 + u;
            rank += (cv[u] > cost || (cv[u] == cost && k < b)) ? 1 : 0;
        }
    }
    if (b < nb) a.order[i0 + rank] = i0 + b;
}


// ---- 5. reverse ----
// REV_GY slot groups per block of beads: the thread of slot group by takes the
// angular slots by, by + REV_GY, ... of its bead, REV_SLOTS of them at a time
constexpr int REV_GY = 8;
constexpr int REV_SLOTS = 2;
// 16-byte key groups of the neighbour's row read together with its header
constexpr int REV_GROUPS = 2;

// key number s (0-based, ascending) of a class part of a row held as 16-byte
// groups: the part inside r_c^A runs up from the row's start, the shell part
// down from its end
__device__ __forceinline__ uint32_t group_key(const uint4 &g, int u, bool down) {
    const int v = down ? 3 - u : u;
    return v == 0 ? g.x : (v == 1 ? g.y : (v == 2 ? g.z : g.w));
}

// slot of `want` in a class part of len keys starting at group g0 of the
// part, or -1; keys at row word 4 + 4 c + u (up) or 4 + A4 - 1 - (4 c + u)
// (down) for group c
__device__ __forceinline__ int find_key_from(const uint32_t *ar, int A4, bool down, int len, int g0, uint32_t want) {
    for (int c = g0; 4 * c < len; ++c) {
        const uint4 g = *reinterpret_cast<const uint4 *>(down ? ar + 4 + A4 - 4 * (c + 1) : ar + 4 + 4 * c);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (4 * c + u < len && group_key(g, u, down) == want) return 4 * c + u;
    }
    return -1;
}

// Reverse entries of up to REV_SLOTS angular slots of bead i: the slot of
// the neighbour j's row that holds i with the opposite image.  The key that
// i has in j's row waits in rev (left by the row kernel); the part of j's
// row of the pair's class (the same in both rows except where rounding puts
// the distance on the two sides of r_c^A) is read with the row's header in
// one round of independent 16-byte loads, and the key is looked up there;
// the rest of a long part, and the other part, only when needed.  Lanes of a
// wave handle consecutive beads at the same slots.  The workgroups of one
// block of beads (its slot groups) are consecutive tiles, kept on one XCD, so
// the neighbours' rows they read stay in that XCD's L2.
__device__ __forceinline__ void nb_reverse_body(const NbArgs &a, int tile) {
    if (build_off(a)) return;
    const int n = a.n;
    const int by = tile % REV_GY;
    const int i = (tile / REV_GY) * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int na = a.cnt[n + i];
    const int A4 = (a.cap_A + 3) & ~3;
    const int nai_i = min(a.cls[i] & 255, na);
    for (int p0 = by; p0 < na; p0 += REV_GY * REV_SLOTS) {
        int p[REV_SLOTS], j[REV_SLOTS];
        uint32_t want[REV_SLOTS];
        bool sh[REV_SLOTS];
#pragma unroll
        for (int k = 0; k < REV_SLOTS; ++k) {
            p[k] = p0 + k * REV_GY;
            const bool v = p[k] < na;
            j[k] = v ? (int)(a.nbr[(size_t)p[k] * n + i] & J_MASK) : 0;
            want[k] = v ? (uint32_t)a.rev[(size_t)p[k] * n + i] : 0u;
            sh[k] = p[k] >= nai_i;
        }
        uint4 hd[REV_SLOTS], g[REV_SLOTS][REV_GROUPS];
#pragma unroll
        for (int k = 0; k < REV_SLOTS; ++k) {
            const uint32_t *ar = a.arow + (size_t)j[k] * (4 + A4);
            hd[k] = *reinterpret_cast<const uint4 *>(ar);
#pragma unroll
            for (int c = 0; c < REV_GROUPS; ++c)
                g[k][c] = 4 * c < A4 ? *reinterpret_cast<const uint4 *>(sh[k] ? ar + 4 + A4 - 4 * (c + 1) : ar + 4 + 4 * c)
                                     : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < REV_SLOTS; ++k) {
            if (p[k] >= na) continue;
            const uint32_t *ar = a.arow + (size_t)j[k] * (4 + A4);
            const int nai_j = (int)hd[k].x, na_j = (int)hd[k].y;
            const int len = sh[k] ? na_j - nai_j : nai_j;
            int found = -1;
#pragma unroll
            for (int c = 0; c < REV_GROUPS; ++c)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (4 * c + u < len && group_key(g[k][c], u, sh[k]) == want[k]) found = 4 * c + u;
            bool shell = sh[k];
            if (found < 0 && len > 4 * REV_GROUPS) found = find_key_from(ar, A4, shell, len, REV_GROUPS, want[k]);
            if (found < 0) {
                shell = !shell;
                found = find_key_from(ar, A4, shell, shell ? na_j - nai_j : nai_j, 0, want[k]);
            }
            const int slot = found < 0 ? -1 : (shell ? nai_j + found : found);
            a.rev[(size_t)p[k] * n + i] = slot < 0 ? -1 : (int32_t)((size_t)slot * n + j[k]);
        }
    }
}

// The reverse search and the processing order in one launch: the first
// nrev workgroups search (nrev is a multiple of 8, so both parts keep the
// XCD-aware tile map), the rest rank their blocks of beads.
__global__ __launch_bounds__(BLOCK) void k_nb_reverse(NbArgs a, int nrev) {
    if ((int)blockIdx.x < nrev) nb_reverse_body(a, xcd_tile(blockIdx.x, nrev));
    else nb_order_body(a, blockIdx.x - nrev, gridDim.x - nrev);
}

// The merge kernel and the pair test of the rebuild gate (the reasoning is
// with FAST_WORDS) in one launch: workgroup 0 runs the merge kernel's work,
// the others one wavefront per listed bead i.  The lanes take the cells around
// i's present position in the build's grid (i has moved, the other beads of a
// pair found this way by less than tau), then the other listed beads.  For
// every pair now inside an interaction cutoff (with the margin: a pair at the
// edge counts as inside) the build-time distance, from the build positions
// with the same image, must lie inside the list cutoff by the margin;
// otherwise the verdict word is set, and a gate of 2 becomes a build.
constexpr int PAIR_TEST_BLOCKS = 64;

__device__ __forceinline__ bool pair_covered(const NbArgs &a, int tp, const float v[3], const float b[3]) {
    const float d2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const float up = 1.0f + PAIR_TEST_MARGIN, down = 1.0f - PAIR_TEST_MARGIN;
    if (!(d2 < a.in2R[tp] * up)) return true;  // outside both interaction cutoffs
    const float b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (!(b2 < a.list2R[tp] * down)) return false;
    if (d2 < a.in2A[tp] * up && !(b2 < a.list2A[tp] * down)) return false;
    return true;
}

__global__ __launch_bounds__(BLOCK) void k_gate_pair_test(KickDriftArgs kd, int nblocks, NbArgs a) {
    if (blockIdx.x == 0) {
        gate_body(kd, nblocks);
        return;
    }
    int32_t *fast = kd.fast;
    // uniform: frozen, no cell data of this call's build yet, or more beads
    // listed than the list holds (then the gate is 1 in any case)
    if ((a.status[0] & FREEZE_MASK) || !fast[2]) return;
    const int cnt = fast[kd.parity];
    if (cnt > FAST_CAP) return;
    const int lane = __lane_id();
    const int nw = (gridDim.x - 1) * (BLOCK / 64);
    const int n = a.n;
    bool bad = false;
    for (int f = (blockIdx.x - 1) * (BLOCK / 64) + (threadIdx.x >> 6); f < cnt; f += nw) {
        const int i = fast[4 + f];
        const float4 pi = a.pos4[i];
        const int ti = min((int)pi.w, a.T - 1);
        const float p[3] = {pi.x, pi.y, pi.z};
        const float r[3] = {a.ref[i], a.ref[n + i], a.ref[2 * n + i]};
        // i's present cell, and the boxes w it has drifted from the build's frame
        int c[3], w[3];
        for (int d = 0; d < 3; ++d) {
            const float L = a.box[d];
            float k = floorf(p[d] / L);
            float x = p[d] - k * L;
            if (x >= L) { x -= L; k += 1.0f; }
            if (x < 0.0f) { x += L; k -= 1.0f; }
            w[d] = (int)k;
            c[d] = cell_coord(x, a.inv_cs[d], a.nc[d]);
        }
        // the (2m+1)^3 <= 125 neighbour cells, two per lane (o = lane, lane + 64):
        // both cells' ranges, then their members four at a time (build records,
        // then present positions), each set of loads issued together; a lane
        // past the offsets has empty ranges, and a short run repeats a member
        const int wx = 2 * a.m[0] + 1, wy = 2 * a.m[1] + 1, wz = 2 * a.m[2] + 1;
        const int W3 = wx * wy * wz;
        int beg[2], end[2], img[2][3];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int o = lane + 64 * h < W3 ? lane + 64 * h : 0;
            const int o3[3] = {o % wx - a.m[0], (o / wx) % wy - a.m[1], o / (wx * wy) - a.m[2]};
            int cc[3];
            for (int d = 0; d < 3; ++d) {
                cc[d] = c[d] + o3[d];
                img[h][d] = w[d];
                if (cc[d] < 0) { cc[d] += a.nc[d]; img[h][d] -= 1; }
                if (cc[d] >= a.nc[d]) { cc[d] -= a.nc[d]; img[h][d] += 1; }
            }
            const int id = cell_index(cc[0], cc[1], cc[2], a.nc);
            beg[h] = a.cell_start[id];
            end[h] = a.cell_start[id + 1];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (lane + 64 * h >= W3) end[h] = beg[h];
        for (int k = 0; beg[0] + k < end[0] || beg[1] + k < end[1]; k += 4) {
            float4 b[2][4], pj[2][4];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = beg[h] + k + u;
                    b[h][u] = a.pos_sorted[q < end[h] ? q : (end[h] > beg[h] ? end[h] - 1 : 0)];
                }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < 4; ++u) pj[h][u] = a.pos4[__float_as_uint(b[h][u].w) & J_MASK];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t tag = __float_as_uint(b[h][u].w);  // index | type << 25
                    const int j = (int)(tag & J_MASK);
                    if (beg[h] + k + u >= end[h] || j == i) continue;
                    const int tp = ti * a.T + min((int)(tag >> CODE_SHIFT), a.T - 1);
                    const float bj[3] = {b[h][u].x, b[h][u].y, b[h][u].z};
                    const float qj[3] = {pj[h][u].x, pj[h][u].y, pj[h][u].z};
                    float v[3], bv[3];
                    for (int d = 0; d < 3; ++d) {
                        const float sh = (float)img[h][d] * a.box[d];
                        v[d] = (qj[d] + sh) - p[d];
                        bv[d] = (bj[d] + sh) - r[d];
                    }
                    if (!pair_covered(a, tp, v, bv)) bad = true;
                }
        }
        // pairs of two listed beads, by the nearest image of their present positions
        for (int g = lane; g < cnt; g += 64) {
            const int j = fast[4 + g];
            if (j == i) continue;
            const float4 pj = a.pos4[j];
            const float qj[3] = {pj.x, pj.y, pj.z};
            const float rj[3] = {a.ref[j], a.ref[n + j], a.ref[2 * n + j]};
            float v[3], bv[3];
            for (int d = 0; d < 3; ++d) {
                const float sh = -rintf((qj[d] - p[d]) / a.box[d]) * a.box[d];
                v[d] = (qj[d] + sh) - p[d];
                bv[d] = (rj[d] + sh) - r[d];
            }
            if (!pair_covered(a, ti * a.T + min((int)pj.w, a.T - 1), v, bv)) bad = true;
        }
    }
    if (bad) fast[3] = 1;  // every writer stores the same value
}

hipError_t launch_gate_pair_test(const KickDriftArgs &k, const NbArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const int nb = (a.n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_gate_pair_test, dim3(1 + PAIR_TEST_BLOCKS), dim3(BLOCK), 0, s, k, nb, a);
    return hipGetLastError();
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
    const size_t lds = row_lds_bytes(a.cap, a.cap_A);
    if (a.T > 1) hipLaunchKernelGGL(k_nb_rows<true>, dim3(a.ncell), dim3(64), lds, s, a);
    else hipLaunchKernelGGL(k_nb_rows<false>, dim3(a.ncell), dim3(64), lds, s, a);
    const int nrev = nbk * REV_GY;
    hipLaunchKernelGGL(k_nb_reverse, dim3(nrev + (a.order ? nbk : 0)), dim3(BLOCK), 0, s, a, nrev);
    return hipGetLastError();
}

// ---- one launch per phase over the builds of many systems ----
// start[kind][r] is the first block of system r for each tile kind (tables of
// n_sys + 1 entries): cells to clear, beads, scan blocks, cells to offset,
// (bead, slot-group) pairs, and runs of cells for the rows.
enum { NB_TILE_CLEAR = 0, NB_TILE_BEAD, NB_TILE_SCANL, NB_TILE_SCANA, NB_TILE_REV, NB_TILE_ROWS, NB_TILES };
static_assert(NB_TILES == NB_BATCH_TILES, "tile kinds of the batched build");
enum { OP_CLEAR, OP_BIN, OP_SCANL, OP_SCANA, OP_FILL, OP_RANK, OP_ORDER, OP_REVERSE };

// the last system whose first block of the given kind is <= blockIdx.x
__device__ __forceinline__ int batch_system(const NbBatchArgs &b, int tile) {
    const int *st = b.start + tile * (b.n_sys + 1);
    int lo = 0, hi = b.n_sys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int OP>
__global__ __launch_bounds__(BLOCK) void k_nb_batch(NbBatchArgs b) {
    constexpr int TILE = OP == OP_CLEAR ? NB_TILE_CLEAR
                         : OP == OP_SCANL ? NB_TILE_SCANL
                         : OP == OP_SCANA ? NB_TILE_SCANA
                         : OP == OP_REVERSE ? NB_TILE_REV
                                            : NB_TILE_BEAD;
    const int *st = b.start + TILE * (b.n_sys + 1);
    const int lo = batch_system(b, TILE);
    const NbArgs &a = b.args[lo];
    const int bx = blockIdx.x - st[lo], gx = st[lo + 1] - st[lo];
    if constexpr (OP == OP_CLEAR) nb_clear_body(a.ncell, a.cell_count, a.status, a.clear_status, a.ctrl, bx, gx);
    if constexpr (OP == OP_BIN) nb_bin_body(a, bx);
    if constexpr (OP == OP_SCANL) scan_local_body(a, bx);
    if constexpr (OP == OP_SCANA) scan_add_body(a, bx);
    if constexpr (OP == OP_FILL) nb_fill_body(a, bx);
    if constexpr (OP == OP_RANK) nb_rank_body(a, bx);
    if constexpr (OP == OP_ORDER) nb_order_body(a, bx, gx);
    if constexpr (OP == OP_REVERSE) {
        nb_reverse_body(a, xcd_tile(bx, gx));
    }
}

// rows of many systems: a cell per workgroup
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_nb_batch_rows(NbBatchArgs b) {
    extern __shared__ __align__(16) uint32_t row_dyn[];
    __shared__ RowsLds L;
    const int *st = b.start + NB_TILE_ROWS * (b.n_sys + 1);
    const int lo = batch_system(b, NB_TILE_ROWS);
    const NbArgs &a = b.args[lo];
    if (build_off(a)) return;  // uniform over the workgroup
    rows_thresholds(a, L);
    const int bx = blockIdx.x - st[lo], gx = st[lo + 1] - st[lo];
    int flags = 0, most = 0, most_a = 0;
    row_cell<true>(a, xcd_tile(bx, gx), L, row_dyn, flags, most, most_a);
    wave_status(a.status, flags, most, most_a);
}

void nb_batch_tiles(const NbArgs &a, int counts[NB_BATCH_TILES]) {
    const int nbk = (a.n + BLOCK - 1) / BLOCK;
    const int cbk = (a.ncell + BLOCK - 1) / BLOCK;
    counts[NB_TILE_CLEAR] = cbk > 0 ? (cbk < 4096 ? cbk : 4096) : 1;
    counts[NB_TILE_BEAD] = nbk;
    counts[NB_TILE_SCANL] = (a.ncell + SCAN_B - 1) / SCAN_B;
    counts[NB_TILE_SCANA] = cbk;
    counts[NB_TILE_REV] = nbk * REV_GY;
    counts[NB_TILE_ROWS] = a.ncell;
}

int nb_row_lds_bytes(int cap, int cap_A) { return row_lds_bytes(cap, cap_A); }

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
    if (totals[NB_TILE_ROWS] > 0)
        hipLaunchKernelGGL(k_nb_batch_rows, dim3(totals[NB_TILE_ROWS]), dim3(64), b.row_bytes, s, b);
    NB_LAUNCH(OP_ORDER, NB_TILE_BEAD)
    NB_LAUNCH(OP_REVERSE, NB_TILE_REV)
#undef NB_LAUNCH
    return hipGetLastError();
}

}  // namespace nep
