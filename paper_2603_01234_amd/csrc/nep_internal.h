// Internal declarations of libnep (HIP, gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nep.h"

namespace nep {

// Descriptor sizes built into the kernels (Sec. II.A): n = 0..8 radial,
// n = 0..6 angular, Chebyshev k = 0..8 for both, l = 1..4.
constexpr int NR = 9;      // radial components
constexpr int NA = 7;      // angular radial functions
constexpr int KB = 9;      // basis functions
constexpr int LM = 24;     // (l, m) pairs for l = 1..4
constexpr int ND = NR + NA * 4;  // 37 descriptor components
constexpr int MAXT = 4;
constexpr int MAXH = 64;
constexpr int BLOCK = 256;
constexpr int TAB_PER_PAIR = NR * KB + NA * KB;  // 81 + 63
constexpr uint32_t J_MASK = 0x1FFFFFFu;
constexpr int CODE_SHIFT = 25;
constexpr float ACCEL = 9.648533212e-5f;  // nm/fs^2 per (eV/nm)/amu
constexpr double KB_EV = 8.617333262e-5;   // Boltzmann constant, eV/K
// per-block partial sums: U, W (9), kinetic energy, radial pairs, angular
// pairs, and (ensemble steps with the HNEMD drive) the driving force (3)
constexpr int NPART = 16;
constexpr int NPART_NVE = 13;   // components the plain and NVE gathers sum
// lanes per bead in the gathers: lane q takes slots q, q + 4, ... of the row,
// and the lane sums are combined by a shuffle butterfly (the same order in the
// single-system, batched MD and fitness gathers)
constexpr int GATHER_LANES = 4;
static_assert(GATHER_LANES * BLOCK <= 1024, "batched MD gather workgroup too large");
// status flags after which the MD kernels do nothing (the lists are invalid)
constexpr int FREEZE_MASK = NEP_FLAG_OVERFLOW_R | NEP_FLAG_OVERFLOW_A | NEP_FLAG_NONFINITE |
                            NEP_FLAG_OUTSIDE_BOX | NEP_FLAG_IMAGE_RANGE | NEP_FLAG_BAD_TYPE;

// Model as held by the library: device copies of the flat parameters and of
// the derived coefficient tables the kernels read.
struct Model {
    int T, H;
    float rcR[MAXT * MAXT], rcA[MAXT * MAXT];
    float *d_params;  // flat layout of nep.h
    float *d_tab;     // [T*T][TAB_PER_PAIR] derived coefficients
    float *d_ann;     // [T][(ND+2)][HP] + 1: w0 transposed, b0, w1 (zero-padded to HP), then b1
    int HP;           // hidden width padded to a built size (8, 16, 32 or 64)
    size_t n_params;
    int device;
    int mfma;         // 1: the network of the single-system fused kernel on the matrix cores
};

// Cutoff tables passed by value.
struct Cut {
    float rcR[MAXT * MAXT], inv_rcR[MAXT * MAXT], rcR2[MAXT * MAXT];
    float rcA[MAXT * MAXT], inv_rcA[MAXT * MAXT], rcA2[MAXT * MAXT];
    // (r_c^A + delta)^2: an angular partial is delivered (zero beyond r_c^A)
    // for every pair its owner finds inside this, and read by the bead at the
    // other end only for a pair it finds inside r_c^A.  The two ends compute
    // the pair's distance with different roundings; delta bounds the
    // difference for coordinates up to the box length (see make_cut).
    float rcA2w[MAXT * MAXT];
};

struct EfvArgs {
    int n, H;
    float box[3];
    const float4 *pos4;     // x, y, z, type
    const uint32_t *nbr;
    const int32_t *rev;
    const int32_t *cnt;
    const float *params;    // flat parameters
    const float *tab;       // derived pair tables
    const float *ann;       // derived network table (see Model::d_ann)
    Cut cut;
    // outputs of the main kernel
    float *U;
    float4 *bvec;           // [n][T][3] radial back-propagation coefficients
    float4 *angbuf;         // [cap_A][n]: slot (q, j) receives dU_i/dr_ij (angular part) from
                            // the neighbour i listed at slot q of row j
    float4 *fown;           // [n] sum_j dU_i/dr_ij (angular)
    const int32_t *freeze;  // MD: status word; the kernel does nothing once FREEZE_MASK is set
    const int32_t *order;   // [n] bead of each thread (null: thread i takes bead i)
};

struct GatherArgs {
    int n;
    float box[3];
    const float4 *pos4;
    const uint32_t *nbr;
    const int32_t *rev;
    const int32_t *cnt;
    const float4 *bvec;
    const float4 *angbuf;
    const float4 *fown;
    Cut cut;
    const float *U;         // site energies (for the energy sum)
    float *F;               // [3][n]
    float *W;               // [9][n] or null
    double *partial;        // [nblocks][16]: U, W(9), K, pairs within r_c^R, pairs within r_c^A
    // fused second half-kick (MD): v = vh + dt/2 a, and the drifted positions
    // (pos4) are written back to x, y, z
    float *v;               // [3][n] or null
    const float *vh;        // [3][n] half-step velocities from the kick-drift kernel
    float *x, *y, *z;
    float half_dt_accel;    // dt/2 * ACCEL
    float inv_mass[MAXT];
    float mass[MAXT];
    const int32_t *freeze;  // MD: status word (see EfvArgs)
    // outside MD: the completeness test of the lists (the reduction flags
    // NEP_FLAG_SKIN once the two largest displacements since the build add up
    // to more than skin_gate)
    const float *ref;       // [3][n] build positions
    float skin_gate;        // 0.99 skin
    float2 *top2;           // [blocks] or null: per-block pairs of that test
    float Fe[3];            // ensemble step with the HNEMD drive: F_e (1/nm)
};

// Cells are numbered tile by tile: tiles of CELL_TILE^3 cells in (z, y, x)
// order, the cells of a tile in (z, y, x) order, the tiles at the upper edges
// cut to the grid.  This is a bijection of the grid onto [0, nx ny nz) under
// which consecutive indices stay close in all three directions, so the beads
// of a workgroup (kept in cell order) lie in a compact block and their
// neighbourhoods overlap in the caches.
constexpr int CELL_TILE = 4;
__device__ __forceinline__ int cell_index(int x, int y, int z, const int nc[3]) {
    constexpr int B = CELL_TILE;
    const int tx = x / B, ty = y / B, tz = z / B;
    const int hx = min(B, nc[0] - tx * B), hy = min(B, nc[1] - ty * B), hz = min(B, nc[2] - tz * B);
    return tz * B * nc[1] * nc[0]            // whole slabs of tiles before
           + ty * B * nc[0] * hz             // whole rows of tiles before, in this slab
           + tx * B * hy * hz                // tiles before, in this row
           + ((z - tz * B) * hy + (y - ty * B)) * hx + (x - tx * B);
}

// XCD-aware tile index: consecutive logical tiles are kept on one XCD (the
// hardware assigns workgroups round-robin over the 8 XCDs, each with its own
// L2), so neighbouring beads share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    constexpr int NX = 8;
    int per = nblocks / NX, rem = nblocks % NX;
    int x = bid % NX, k = bid / NX;
    // XCD x owns logical tiles [start_x, start_x + per + (x < rem))
    int start = x * per + (x < rem ? x : rem);
    int cnt_x = per + (x < rem ? 1 : 0);
    if (k < cnt_x) return start + k;
    return bid;  // not reached for a full grid
}

__device__ __forceinline__ void decode(uint32_t e, int &j, int &nx, int &ny, int &nz) {
    j = (int)(e & J_MASK);
    int c = (int)(e >> CODE_SHIFT);
    int c5 = c / 5;
    nx = c - 5 * c5 - 2;
    int c25 = c5 / 5;
    ny = c5 - 5 * c25 - 2;
    nz = c25 - 2;
}

// Chebyshev polynomials T_0..T_8 and U_0..U_7 (for T_k' = k U_{k-1}).
__device__ __forceinline__ void cheb_T(float x, float T[KB]) {
    T[0] = 1.0f;
    T[1] = x;
    float x2 = 2.0f * x;
#pragma unroll
    for (int k = 2; k < KB; ++k) T[k] = x2 * T[k - 1] - T[k - 2];
}
__device__ __forceinline__ void cheb_U(float x, float Uc[KB - 1]) {
    Uc[0] = 1.0f;
    float x2 = 2.0f * x;
    Uc[1] = x2;
#pragma unroll
    for (int k = 2; k < KB - 1; ++k) Uc[k] = x2 * Uc[k - 1] - Uc[k - 2];
}

// Real solid-harmonic polynomials P_lm(u), l = 1..4, on the unit sphere.  With
// the weights N2_lm, sum_m N2_lm P_lm(u) P_lm(v) = (2l+1)/(4 pi) P_l(u.v), so
// sum_m N2 A_lm^2 equals the complex sum of Eq. 4.  The visitors below walk the
// 24 terms one at a time (value, and for the force also grad_u P), so no
// 24-wide temporaries stay live next to the 168 accumulators.
template <int IDX>
__device__ __forceinline__ void acc_lm(float P, const float g[NA], float A[NA][LM]) {
#pragma unroll
    for (int q = 0; q < NA; ++q) A[q][IDX] += g[q] * P;
}

// A_{n,lm} += g_n P_lm(u)
__device__ __forceinline__ void accumulate_harmonics(float x, float y, float z, const float g[NA],
                                                     float A[NA][LM]) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    acc_lm<0>(x, g, A);
    acc_lm<1>(y, g, A);
    acc_lm<2>(z, g, A);
    acc_lm<3>(x * y, g, A);
    acc_lm<4>(y * z, g, A);
    acc_lm<5>(x * z, g, A);
    acc_lm<6>(x2 - y2, g, A);
    acc_lm<7>(3.0f * z2 - 1.0f, g, A);
    const float a = 3.0f * x2 - y2, b = 5.0f * z2 - 1.0f, c = x2 - 3.0f * y2, d = x2 - y2;
    acc_lm<8>(y * a, g, A);
    acc_lm<9>(x * y * z, g, A);
    acc_lm<10>(y * b, g, A);
    acc_lm<11>(z * (5.0f * z2 - 3.0f), g, A);
    acc_lm<12>(x * b, g, A);
    acc_lm<13>(z * d, g, A);
    acc_lm<14>(x * c, g, A);
    const float e = 7.0f * z2 - 1.0f, f = 7.0f * z2 - 3.0f;
    acc_lm<15>(x * y * d, g, A);
    acc_lm<16>(y * z * a, g, A);
    acc_lm<17>(x * y * e, g, A);
    acc_lm<18>(y * z * f, g, A);
    acc_lm<19>((35.0f * z2 - 30.0f) * z2 + 3.0f, g, A);
    acc_lm<20>(x * z * f, g, A);
    acc_lm<21>(d * e, g, A);
    acc_lm<22>(x * z * c, g, A);
    acc_lm<23>(x2 * x2 - 6.0f * x2 * y2 + y2 * y2, g, A);
}

// one term of the pair partial: B = sum_n D_n g_n, V += B grad_u P, and
// sig_n += D_n P for the radial part s = sum_n g_n' sig_n (one FMA per term
// fewer than summing B' = sum_n D_n g_n' per term)
template <int IDX>
__device__ __forceinline__ void force_lm(float P, float Gx, float Gy, float Gz, const float D[NA][LM],
                                         const float g[NA], float &vx, float &vy, float &vz, float sig[NA]) {
    float B = 0.0f;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        B += D[q][IDX] * g[q];
        sig[q] += D[q][IDX] * P;
    }
    vx += B * Gx;
    vy += B * Gy;
    vz += B * Gz;
}

__device__ __forceinline__ void force_harmonics(float x, float y, float z, const float D[NA][LM],
                                                const float g[NA], const float gp[NA], float &s,
                                                float &vx, float &vy, float &vz) {
    float sig[NA] = {0.0f, 0.0f, 0.0f, 0.0f};
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, yz = y * z, xz = x * z, xyz = xy * z;
    force_lm<0>(x, 1.0f, 0.0f, 0.0f, D, g, vx, vy, vz, sig);
    force_lm<1>(y, 0.0f, 1.0f, 0.0f, D, g, vx, vy, vz, sig);
    force_lm<2>(z, 0.0f, 0.0f, 1.0f, D, g, vx, vy, vz, sig);
    force_lm<3>(xy, y, x, 0.0f, D, g, vx, vy, vz, sig);
    force_lm<4>(yz, 0.0f, z, y, D, g, vx, vy, vz, sig);
    force_lm<5>(xz, z, 0.0f, x, D, g, vx, vy, vz, sig);
    force_lm<6>(x2 - y2, 2.0f * x, -2.0f * y, 0.0f, D, g, vx, vy, vz, sig);
    force_lm<7>(3.0f * z2 - 1.0f, 0.0f, 0.0f, 6.0f * z, D, g, vx, vy, vz, sig);
    const float d = x2 - y2, b51 = 5.0f * z2 - 1.0f;
    force_lm<8>(y * (3.0f * x2 - y2), 6.0f * xy, 3.0f * d, 0.0f, D, g, vx, vy, vz, sig);
    force_lm<9>(xyz, yz, xz, xy, D, g, vx, vy, vz, sig);
    force_lm<10>(y * b51, 0.0f, b51, 10.0f * yz, D, g, vx, vy, vz, sig);
    force_lm<11>(z * (5.0f * z2 - 3.0f), 0.0f, 0.0f, 15.0f * z2 - 3.0f, D, g, vx, vy, vz, sig);
    force_lm<12>(x * b51, b51, 0.0f, 10.0f * xz, D, g, vx, vy, vz, sig);
    force_lm<13>(z * d, 2.0f * xz, -2.0f * yz, d, D, g, vx, vy, vz, sig);
    force_lm<14>(x * (x2 - 3.0f * y2), 3.0f * d, -6.0f * xy, 0.0f, D, g, vx, vy, vz, sig);
    const float a3 = 3.0f * x2 - y2, c3 = x2 - 3.0f * y2;
    const float e = 7.0f * z2 - 1.0f, f = 7.0f * z2 - 3.0f, h = 21.0f * z2 - 3.0f;
    force_lm<15>(xy * d, y * a3, x * c3, 0.0f, D, g, vx, vy, vz, sig);
    force_lm<16>(yz * a3, 6.0f * xyz, 3.0f * z * d, y * a3, D, g, vx, vy, vz, sig);
    force_lm<17>(xy * e, y * e, x * e, 14.0f * xyz, D, g, vx, vy, vz, sig);
    force_lm<18>(yz * f, 0.0f, z * f, y * h, D, g, vx, vy, vz, sig);
    force_lm<19>((35.0f * z2 - 30.0f) * z2 + 3.0f, 0.0f, 0.0f, z * (140.0f * z2 - 60.0f), D, g, vx, vy, vz,
                 sig);
    force_lm<20>(xz * f, z * f, 0.0f, x * h, D, g, vx, vy, vz, sig);
    force_lm<21>(d * e, 2.0f * x * e, -2.0f * y * e, 14.0f * z * d, D, g, vx, vy, vz, sig);
    force_lm<22>(xz * c3, 3.0f * z * d, -6.0f * xyz, x * c3, D, g, vx, vy, vz, sig);
    force_lm<23>(x2 * x2 - 6.0f * x2 * y2 + y2 * y2, 4.0f * x * c3, 4.0f * y * (y2 - 3.0f * x2), 0.0f, D, g,
                 vx, vy, vz, sig);
#pragma unroll
    for (int q = 0; q < NA; ++q) s += gp[q] * sig[q];
}

// cos(pi t) and sin(pi t) for 0 <= t <= 1 with the hardware instructions,
// whose argument is in revolutions (cos(2 pi x))
__device__ __forceinline__ float cos_pi(float t) { return __builtin_amdgcn_cosf(0.5f * t); }
__device__ __forceinline__ float sin_pi(float t) { return __builtin_amdgcn_sinf(0.5f * t); }

// branch-free tanh: sign(x) (1 - 2 / (exp(2|x|) + 1)); absolute error ~1e-7,
// saturates to +-1 without overflow (exp -> inf gives 2/inf = 0)
__device__ __forceinline__ float tanh_nobranch(float x) {
    const float e = __expf(2.0f * fabsf(x));
    // hardware reciprocal (1 ulp); e = inf gives exactly 1
    const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
    return copysignf(t, x);
}

__device__ __forceinline__ int lm_l(int lm) { return lm < 3 ? 1 : lm < 8 ? 2 : lm < 15 ? 3 : 4; }

// launchers (defined in the .hip files)
hipError_t launch_pack(int n, int T, const float *x, const float *y, const float *z, const uint8_t *type,
                       float4 *pos4, hipStream_t s);
// mfma: the network on the matrix cores (one type, HP 16, 32 or 64; see
// efv_main_mfma_supported)
hipError_t launch_efv_main(int T, int HP, const EfvArgs &a, size_t lds_bytes, hipStream_t s, bool mfma = false);
bool efv_main_mfma_supported(int T, int HP);
// md: 0 plain evaluation, 1 NVE step (second half-kick and commit fused in),
// 2 ensemble step (forces, per-bead virial and, with hn, the HNEMD drive; the
// kick follows in the ensemble kernels)
hipError_t launch_efv_gather(int T, bool virial, int md, bool hn, const GatherArgs &a, hipStream_t s);
// top2 (optional): the gather blocks' pairs of the rebuild test; the reduction
// sets NEP_FLAG_SKIN in skin_status when they call for a rebuild
hipError_t launch_reduce(const double *partial, int nblocks, double *E_tot, double *W_tot,
                         double *K_tot, double *E_slot, double *K_slot, double *W_slot, double *counts,
                         const int32_t *status, int32_t *ctrl, int next_gate, const float2 *top2,
                         float skin_gate, float reach, int32_t *skin_status, hipStream_t s);
struct NbArgs {
    int n, cap, cap_A;
    float box[3];
    int pbc[3];
    int nc[3], m[3];
    float inv_cs[3];
    float list2R[MAXT * MAXT], list2A[MAXT * MAXT];
    float in2R[MAXT * MAXT], in2A[MAXT * MAXT];  // squared interaction cutoffs (row classes)
    int T;
    const float *x, *y, *z;
    float *x_mut, *y_mut, *z_mut;  // same arrays, written only when wrap is set
    const uint8_t *type;
    float4 *pos4;
    int32_t *cell_id, *cell_count, *cell_start, *cell_cursor, *cell_list, *scan_tmp;
    int32_t *cell_xyz;   // [ncell] grid coordinates of each cell, x | y << 10 | z << 20 (nc <= 1023)
    int32_t *cell_tmp;   // [n] cell members in atomic (arbitrary) order
    float4 *pos_sorted;  // [n] positions in cell order; w = bits of (index | type << 25)
    int32_t *cls;        // [n] entries inside r_c^A | entries inside r_c^R (radial-only) << 8
    float cull2;         // cells whose gap exceeds this squared distance are skipped
    uint32_t *arow;      // [n][4 + A4] (A4: cap_A rounded up to a multiple of 4) angular sort
                         // keys, row-major: header (entries inside r_c^A, angular entries, 0, 0),
                         // then the keys inside r_c^A up from word 4 and the shell's down from
                         // the row's end
    uint32_t *nbr;
    int32_t *rev, *cnt;
    float *ref;
    int32_t *status;
    int32_t *ctrl;     // MD: [0] rebuild gate set by the preceding reduction, [1] rebuild
                       // count; null: build unconditionally
    int ncell;
    int clear_status;  // 1: a fresh build resets the status word
    int wrap;          // 1: wrap periodic coordinates into [0, L) and write them back first
    int32_t *order;    // [n] or null: processing order for the fused kernel, written from the row counts
    int from_pos4;     // 1 (MD): positions come from pos4 and are wrapped there, x/y/z are untouched
    int skip_clear;    // 1 (MD): the drift kernel of the step already zeroed the cell counts, so no
                       // clearing launch; the bin phase then counts the rebuild in ctrl[1]
    int32_t *fast;     // MD with the pair test (see FAST_WORDS) or null: the bin phase marks the
                       // cell data as this call's
};
hipError_t launch_build(const NbArgs &a, hipStream_t s);

// Builds of many systems, one launch per phase: args[r] as for launch_build
// (systems with n > 0); start holds the tables of first blocks written by
// the caller from nb_batch_tiles; totals are the last entries of the tables.
constexpr int NB_BATCH_TILES = 6;
struct NbBatchArgs {
    int n_sys;
    const NbArgs *args;
    const int *start;     // [NB_BATCH_TILES][n_sys + 1]
    int row_bytes;        // largest nb_row_lds_bytes over the systems
};
void nb_batch_tiles(const NbArgs &a, int counts[NB_BATCH_TILES]);
// LDS bytes the row kernel takes for a row of the given capacities
int nb_row_lds_bytes(int cap, int cap_A);
hipError_t launch_build_batch(const NbBatchArgs &b, const int totals[NB_BATCH_TILES], hipStream_t s);

// zeroes the status word and, when given, the MD control words [4] (the
// rebuild gate ctrl[0] is set to gate0)
hipError_t launch_clear_status(int32_t *status, int32_t *ctrl, int gate0, hipStream_t s,
                               int32_t *fast = nullptr);

// First half of a velocity-Verlet step.  Reads x, v, F; writes the half-step
// velocities to vh and the drifted (and strained) positions to pos4, leaving
// x and v to the gather kernel that completes the step.  Each workgroup leaves
// the largest and second largest displacement of its beads in top2 for the
// rebuild test below.
struct KickDriftArgs {
    int n;
    const float *x, *y, *z;
    const float *v;         // [3][n]
    float *vh;              // [3][n]
    const float *F;         // [3][n]
    const uint8_t *type;
    float4 *pos4;
    float *ref;             // [3][n] positions at the last build (strained in place)
    float half_dt_accel;    // dt/2 * ACCEL
    float dt;
    float inv_mass[MAXT];
    float lam[3];           // affine scale factors of this step
    float box[3];           // box after the strain
    int pbc[3];
    int T;                  // number of types (type values are clamped below it)
    float skin_gate;        // 0.99 skin: a rebuild is due once the two largest
                            // displacements since the build add up to more
    float reach;            // largest r_c + skin (the affine-shrink term of the test)
    float2 *top2;           // [blocks] per-block largest and second largest squared displacement
    int32_t *status;        // [3] holds sigma (updated by the merge kernel)
    int32_t *ctrl;          // ctrl[0]: rebuild gate
    int32_t *cell_count;    // or null: cell counts of the step's build, zeroed here
    int ncell;
    // or null: the previous step's block partials, reduced by the merge kernel
    // (in place of a reduction launch of their own) into the slots below
    const double *prev_partial;
    int prev_blocks;
    double *pre;            // [drift workgroups][NPART]: the drift workgroup's sums of consecutive
                            // ranges of those partials, which the merge kernel then reduces
    double *prev_E, *prev_K, *prev_W, *counts;
    int next_gate;          // the schedule's gate for this step's build
    int32_t *fast;          // or null: the pair test's words (FAST_WORDS); beads whose squared
    float tau2;             // displacement reaches tau2 are listed for it
    int parity;             // which of the two list counters this step's drift uses
    int rebuild_every;      // with fast: the largest number of steps a list serves once the call
                            // has built one (ctrl[3] counts them; before, the schedule's gate)
};
// the drift, then one workgroup that merges the blocks' pairs and switches
// the rebuild gate on when they call for a rebuild
// with gate = false the merge kernel is left to launch_gate_pair_test
hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t s, bool gate = true);
// the merge kernel of the drift (k) and, in the same launch, the pair test of
// the rebuild gate (see FAST_WORDS) on the build's cell data (a)
hipError_t launch_gate_pair_test(const KickDriftArgs &k, const NbArgs &a, hipStream_t s);

// ---- the rebuild test ----
// Gate values (ctrl[0]): 0 no build, 1 build, 2 the pair test decides (the
// build runs only if the test turns the gate to 1).
//
// The pair test.  Call tau = skin_gate / 2.  Two beads that have both moved
// less than tau since the build have a pair distance changed by less than
// skin_gate, so such a pair is covered by the lists.  Every other pair has a
// bead that moved at least tau; the drift lists those beads, and when the
// two-largest test fires the check kernel looks at every pair of a listed
// bead that is now inside an interaction cutoff: it must have been inside the
// list cutoff at the build (then both rows hold it), with a relative margin
// for the rounding of the list predicate.  Candidates are found through the
// build's cell data (a bead that moved less than tau is still within reach of
// the cells it was binned in) and, for pairs of two listed beads, through the
// list itself.  The test is used only within an MD call whose lists were built
// by that call, in a fully periodic box with every side at least three times
// the list reach, without strain or barostat; otherwise the gate is 1.
// The check runs beside the merge kernel (one launch), whenever beads are
// listed, and leaves its verdict for the build to combine with the gate.
// Words: [0], [1] beads listed by the drift of steps of even and odd parity
// (the drift clears the other one for the next step), [2] cell data of this
// call's build present, [3] a listed pair came from outside the lists (cleared
// by the drift), then the list.
constexpr int FAST_CAP = 1024;
constexpr int FAST_WORDS = 4 + FAST_CAP;
constexpr float PAIR_TEST_MARGIN = 1e-5f;
// A pair's distance changes by at most |d_i| + |d_j| (d: displacements since
// the build; periodic images move with their bead), which is at most the sum
// of the two largest displacements of the system.  While that sum stays below
// the skin no pair can have come from beyond r_c + skin to inside r_c, so the
// lists are complete.  The 1% margin covers the rounding of the list predicate.

// (a, b) = largest and second largest of a set of values; merged with (a2, b2)
__device__ __forceinline__ void top2_merge(float &a, float &b, float a2, float b2) {
    const float hi = fmaxf(a, a2), lo = fminf(a, a2);
    b = fmaxf(lo, fmaxf(b, b2));
    a = hi;
}

// the pair of the whole workgroup (every thread calls it; valid in thread 0)
__device__ __forceinline__ float2 block_top2(float a, float b) {
    __shared__ float2 wtop[BLOCK / 64];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) top2_merge(a, b, __shfl_xor(a, o), __shfl_xor(b, o));
    if (__lane_id() == 0) wtop[threadIdx.x >> 6] = make_float2(a, b);
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < BLOCK / 64; ++w) top2_merge(a, b, wtop[w].x, wtop[w].y);
    return make_float2(a, b);
}

// the pair of n per-workgroup pairs, merged by one workgroup (valid in thread 0)
__device__ __forceinline__ float2 merge_top2(const float2 *top2, int n) {
    float a = 0.0f, b = 0.0f;
    for (int k = threadIdx.x; k < n; k += BLOCK) top2_merge(a, b, top2[k].x, top2[k].y);
    return block_top2(a, b);
}

// Fixed-order FP64 reduction of the gather's block partials by one workgroup
// of BLOCK threads (every thread calls it).  In MD mode (ctrl given) it counts
// the completed step in ctrl[2] and sets the rebuild gate ctrl[0] to the
// schedule's next_gate (the next drift may still switch it on).  Once the
// status carries a freeze flag nothing but the gate is written.
// With NP = NPART (ensemble steps) it also leaves, in ens, the mean driving
// force (ens[0..2] = the block sums of components 13..15 times inv_n) and the
// step's total virial (ens[3..11]).
template <int NP = NPART_NVE>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ partial, int nblocks, double *E_tot,
                                                double *W_tot, double *K_tot, double *E_slot, double *K_slot,
                                                double *W_slot, double *counts, const int32_t *status,
                                                int32_t *ctrl, int next_gate, double *ens = nullptr,
                                                double inv_n = 0.0) {
    __shared__ double wsum[NP][BLOCK / 64];
    __shared__ double tot[NP];
    double acc[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) acc[c] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += BLOCK) {
#pragma unroll
        for (int c = 0; c < NP; ++c) acc[c] += partial[(size_t)b * NPART + c];
    }
    // a butterfly within each wave (every lane ends with the same sum), then
    // the waves in order
#pragma unroll
    for (int c = 0; c < NP; ++c) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc[c] += __shfl_xor(acc[c], o);
    }
    if (__lane_id() == 0) {
#pragma unroll
        for (int c = 0; c < NP; ++c) wsum[c][threadIdx.x >> 6] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < NP) {
        double v = wsum[threadIdx.x][0];
#pragma unroll
        for (int w = 1; w < BLOCK / 64; ++w) v += wsum[threadIdx.x][w];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    const int st0 = status ? status[0] : 0;
    if (threadIdx.x == 0 && ctrl) {
        ctrl[0] = next_gate;
        if (!(st0 & FREEZE_MASK)) ctrl[2] += 1;
    }
    if (st0 & FREEZE_MASK) return;
    if (threadIdx.x == 0) {
        if (E_tot) *E_tot = tot[0];
        if (E_slot) *E_slot = tot[0];
        if (K_tot) *K_tot = tot[10];
        if (K_slot) *K_slot = tot[10];
        if (counts) {
            counts[0] += tot[11];
            counts[1] += tot[12];
        }
    }
    if (W_tot && threadIdx.x < 9) W_tot[threadIdx.x] = tot[1 + threadIdx.x];
    if (W_slot && threadIdx.x < 9) W_slot[threadIdx.x] = tot[1 + threadIdx.x];
    if constexpr (NP == NPART) {
        if (ens && threadIdx.x < 3) ens[threadIdx.x] = tot[13 + threadIdx.x] * inv_n;
        if (ens && threadIdx.x < 9) ens[3 + threadIdx.x] = tot[1 + threadIdx.x];
    }
}

// The compression factor sigma of the lists (status[3], float bits): the
// product over the steps since the build of min(1, smallest scale factor of
// the step).  Each periodic image moves affinely with the box, so a pair at
// r >= r_c + skin at the build is now at least sigma (r_c + skin) minus the
// non-affine displacements of its two beads.  A word that is not a factor in
// (0, 1] (lists from before this convention) counts as 0, which asks for a
// rebuild.
__device__ __forceinline__ float sigma_of(int32_t w) {
    const float s = __int_as_float(w);
    return (s > 0.0f && s <= 1.0f) ? s : 0.0f;
}
constexpr int32_t SIGMA_ONE = 0x3f800000;  // bits of 1.0f

// whether a pair of squared non-affine displacements, together with the
// affine shrink (1 - sigma) reach (reach = largest r_c + skin), calls for a
// rebuild
__device__ __forceinline__ bool past_skin(float2 t, float skin_gate, float shrink = 0.0f) {
    return sqrtf(t.x) + sqrtf(t.y) + shrink > skin_gate;
}

// The merge kernel's work (one workgroup): the previous step's reduction
// (second level, over the drift workgroups' sums; it also sets the gate to the
// schedule), then the rebuild test over the pairs of the drift's workgroups
// with the affine shrink of the lists' compression factor sigma, updated by
// this step's scale factors (and reset to 1 when the step rebuilds).  When the
// test fires and the pair test can decide instead, the gate is 2.
__device__ __forceinline__ void gate_body(const KickDriftArgs &a, int nblocks) {
    // the words the decision reads, loaded before the reductions so that
    // their latency overlaps them (no other workgroup writes them meanwhile)
    int32_t st3 = 0, age = -1, cells = 0, listed = 0;
    if (threadIdx.x == 0) {
        st3 = a.status[3];
        if (a.fast) {
            age = a.ctrl[3];
            cells = a.fast[2];
            listed = a.fast[a.parity];
        }
    }
    if (a.prev_partial)
        reduce_partials(a.pre, nblocks, nullptr, nullptr, nullptr, a.prev_E, a.prev_K, a.prev_W, a.counts,
                        a.status, a.ctrl, a.next_gate);
    if (a.status[0] & FREEZE_MASK) return;
    const float2 t = merge_top2(a.top2, nblocks);
    if (threadIdx.x == 0) {
        const float lmin = fminf(1.0f, fminf(a.lam[0], fminf(a.lam[1], a.lam[2])));
        const float sig = sigma_of(st3) * lmin;
        // with the pair test, the schedule counts the steps the lists have
        // served since this call built them (ctrl[3] >= 0 once it has)
        if (a.fast && age >= 0) {
            a.ctrl[3] = age + 1;
            a.ctrl[0] = age + 1 >= a.rebuild_every ? 1 : 0;
        }
        if (a.ctrl[0] != 1 && past_skin(t, a.skin_gate, (1.0f - sig) * a.reach)) {
            const bool pair_test = a.fast && sig == 1.0f && cells != 0 && listed <= FAST_CAP;
            a.ctrl[0] = pair_test ? 2 : 1;
        }
        a.status[3] = a.ctrl[0] ? SIGMA_ONE : __float_as_int(sig);
    }
}

// First half-kick and drift of bead i (kick k = dt/2 ACCEL / m of its type):
// half-step velocity to vh, new position (scaled by lam) to pos4, build
// reference scaled in place.  Returns the squared distance from the bead's
// build position.  Split into the reads and the rest, so that a caller can
// issue the reads before a test that decides whether to write.
struct BeadIn {
    float x, y, z, vx, vy, vz, fx, fy, fz, rx, ry, rz;
};
__device__ __forceinline__ BeadIn kick_drift_read(int i, int n, const float *x, const float *y, const float *z,
                                                  const float *v, const float *F, const float *ref) {
    return BeadIn{x[i],     y[i],         z[i],         v[i],   v[n + i],     v[2 * n + i],
                  F[i],     F[n + i],     F[2 * n + i], ref[i], ref[n + i],   ref[2 * n + i]};
}
__device__ __forceinline__ float kick_drift_write(const BeadIn &b, int i, int n, int t, float k, float dt, float l0,
                                                  float l1, float l2, float *vh, float4 *pos4, float *ref) {
    const float vx = b.vx + k * b.fx;
    const float vy = b.vy + k * b.fy;
    const float vz = b.vz + k * b.fz;
    vh[i] = vx;
    vh[n + i] = vy;
    vh[2 * n + i] = vz;
    const float px = (b.x + dt * vx) * l0;
    const float py = (b.y + dt * vy) * l1;
    const float pz = (b.z + dt * vz) * l2;
    const float rx = b.rx * l0, ry = b.ry * l1, rz = b.rz * l2;
    ref[i] = rx;
    ref[n + i] = ry;
    ref[2 * n + i] = rz;
    pos4[i] = make_float4(px, py, pz, (float)t);
    const float dx = px - rx, dy = py - ry, dz = pz - rz;
    return dx * dx + dy * dy + dz * dz;
}
__device__ __forceinline__ float kick_drift_bead(int i, int n, int t, float k, float dt, float l0, float l1,
                                                 float l2, const float *x, const float *y, const float *z,
                                                 const float *v, float *vh, const float *F, float4 *pos4,
                                                 float *ref) {
    return kick_drift_write(kick_drift_read(i, n, x, y, z, v, F, ref), i, n, t, k, dt, l0, l1, l2, vh, pos4, ref);
}


// ---- ensemble steps (thermostat, per-call barostat, HNEMD drive) ----
// ens (doubles, workspace): [0..2] mean driving force of the step, [3..11]
// the step's total virial, [12] the thermostat factor lambda, [13..15] the
// running sum of the diagonal pressure over the call's steps.
constexpr int ENS_DOUBLES = 16;
struct EnsArgs {
    int n, T;
    const int32_t *status;  // freeze test
    int32_t *ctrl;          // MD control words (completed-step count, gate)
    // after the gather
    const double *partial;  // gather blocks [nblocks][NPART]
    int nblocks;
    double *E_slot, *W_slot, *counts;
    int next_gate;
    // finish: drive without its mean, second half-kick, commit
    float *F;               // [3][n] total force (in: with the drive, out: mean removed)
    const float4 *pos4;
    float *x, *y, *z, *v;
    const float *vh;
    const uint8_t *type;
    const float *Wb;        // [9][n] per-bead virial of the step (HNEMD) or null
    int hn;                 // 1: remove the mean drive and sum the heat current
    float half_dt_accel;
    float inv_mass[MAXT], mass[MAXT];
    double *partial2;       // finish blocks [nb][8]: K, Kxx, Kyy, Kzz, Jx, Jy, Jz
    int nb2;
    // thermostat and traces
    int thermostat;         // 0 none, 1 Berendsen, 2 Bussi
    double T_target, tau_T, dt, kB;
    const double *noise;    // [2] this step's R and S (Bussi) or null
    double *K_slot, *J_slot;
    double volume;          // box volume after this step's drift (nm^3)
    double *ens;
    // constrained bead centres of mass (n_groups 0: none)
    int n_groups;
    const int32_t *group_start;
    double *F_sum, *W_sum;  // [3][n_groups], [9][n_groups]
};
hipError_t launch_ensemble_step(const EnsArgs &e, hipStream_t s);
// the constraint projection of F alone (start of a call; nothing accumulated)
hipError_t launch_constraint_project(const EnsArgs &e, hipStream_t s);
hipError_t launch_ensemble_clear(double *ens, hipStream_t s);

// ---- SNES on the device (the training loop around the fitness kernel) ----
constexpr int DERIVE_MAX = 64;   // models per derivation launch
struct DeriveArgs {
    int T, H, HP;
    size_t n_params;
    const float *params;         // [n_models][n_params] flat vectors (layout of nep.h)
    float *tab[DERIVE_MAX];      // each model's pair tables
    float *ann[DERIVE_MAX];      // each model's network table
    float *flat[DERIVE_MAX];     // each model's copy of the flat vector
};
hipError_t launch_derive_tables(const DeriveArgs &a, int n_models, hipStream_t s);
hipError_t launch_snes_sample(int pop, size_t dim, const float *mu, const float *sigma, const float *s, float *z,
                              hipStream_t st);
hipError_t launch_snes_update(int pop, size_t dim, const float *s, const float *z, const double *rmse,
                              const nep_snes_params &h, float *mu, float *sigma, double *loss, int32_t *order,
                              hipStream_t st);

// ---- batched evaluation (fitness loop) ----
struct SysDesc {           // one structure of the batch
    int n;
    int label_off;         // first row of the structure in the concatenated force labels
    float box[3];
    const float *x, *y, *z;
    const uint8_t *type;
    const uint32_t *nbr;
    const int32_t *rev, *cnt;
};
struct ModelDesc {         // one candidate parameter set
    const float *tab, *ann;
};
struct BatchArgs {
    int n_items;
    const int4 *items;     // schedule order: (model, system, index in the caller's list, 0)
    const SysDesc *sys;
    const ModelDesc *mod;
    Cut cut;               // shared by every candidate (the lists are shared)
    int *counter;          // work-queue head, zeroed before the launch
    char *scratch;         // per-workgroup intermediates, scratch_stride bytes each
    size_t scratch_stride;
    int nmax, capAmax;     // largest structure and angular capacity in the batch
    const double *F_ref;   // [sum_s n_s][3] or null
    double *records;       // [n_items][12] by list index
    float *F_out;          // [sum over items of n][3] or null
    const int64_t *F_off;  // first row of each item in F_out, by list index
};
hipError_t launch_efv_batch(int T, int HP, int BS, const BatchArgs &b, int grid, hipStream_t s);
int batch_occupancy(int T, int HP, int BS);
hipError_t launch_batch_rmse(int n_models, int n_items, const int4 *list, const SysDesc *sys,
                             const double *records, const double *E_ref, const double *W_ref, double *rmse,
                             double *item_out, hipStream_t s);


// ---- many replicas, one MD step each (served form) ----
struct RepDesc {
    int n;
    float skin_gate;       // 0.99 skin (the rebuild test above)
    float2 *top2;          // [tiles] per-tile pairs of the rebuild test (replica's workspace)
    float box[3];
    float *x, *y, *z, *v, *F, *U;
    const uint8_t *type;
    const uint32_t *nbr;
    const int32_t *rev, *cnt;
    float *ref;
    int32_t *status;       // [3]: sigma (reset to 1 when the step rebuilds)
    // the replica's own workspace
    float4 *pos4, *bvec, *angbuf, *fown;
    float *vh;
    double *partial;       // [tiles][2]: potential and kinetic energy per tile
    const int32_t *order;  // [n] or null: processing order of the fused kernel, written by the builds
    float reach;           // largest r_c + skin (affine-shrink term of the rebuild test)
};
struct MdBatchArgs {
    int n_rep, n_tiles, T;
    const RepDesc *rep;
    const int *tile_start; // [n_rep + 1] first tile of every replica
    int *gate;             // [n_rep] rebuild gate, set by the drift
    float half_dt_accel, dt;
    float inv_mass[MAXT], mass[MAXT];
    Cut cut;
    const float *tab, *ann;
    double *E_pot, *E_kin; // [n_rep] or null
    int32_t *status_out;   // [n_rep][4] copies of the status words after the step
};
hipError_t launch_kick_drift_batch(const MdBatchArgs &b, hipStream_t s);
// fused kernel, gather (second half-kick) and per-replica energy sums
hipError_t launch_efv_md_batch(int T, int HP, const MdBatchArgs &b, hipStream_t s);


// In-place reordering of a system's per-bead arrays: new position s takes old
// bead src[s] for x, y, z, type and, when given, v, F, U and perm.
struct PermuteArgs {
    int n;
    const int32_t *src;
    float *x, *y, *z;
    uint8_t *type;
    float *v, *F, *U;   // [3][n], [3][n], [n] or null
    int32_t *perm;      // [n] or null
    float *tmp;         // [12][n] floats and [n] bytes
};
hipError_t launch_permute(const PermuteArgs &a, hipStream_t s);

}  // namespace nep
