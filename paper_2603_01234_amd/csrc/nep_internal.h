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
constexpr int TAB_PER_PAIR = NR * KB + NA * KB + NA * (KB - 1);  // 81 + 63 + 56
constexpr uint32_t J_MASK = 0x1FFFFFFu;
constexpr int CODE_SHIFT = 25;
constexpr float ACCEL = 9.648533212e-5f;  // nm/fs^2 per (eV/nm)/amu
// per-block partial sums: U, W (9), kinetic energy, radial pairs, angular pairs;
// slots 13..15 of each block hold maxima for the rebuild prediction
constexpr int NPART = 13;
constexpr int NMAX = 3;
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
    size_t n_params;
    int device;
};

// Cutoff tables passed by value.
struct Cut {
    float rcR[MAXT * MAXT], inv_rcR[MAXT * MAXT], rcR2[MAXT * MAXT];
    float rcA[MAXT * MAXT], inv_rcA[MAXT * MAXT], rcA2[MAXT * MAXT];
};

struct EfvArgs {
    int n, H;
    float box[3];
    const float4 *pos4;     // x, y, z, type
    const uint32_t *nbr;
    const int32_t *cnt;
    const float *params;    // flat parameters
    const float *tab;       // derived tables
    Cut cut;
    // outputs of the main kernel
    float *U;
    float4 *bvec;           // [n][T][3] radial back-propagation coefficients
    float4 *angbuf;         // [cap_A][n] dU_i/dr_ij angular part
    float4 *fown;           // [n] sum_j dU_i/dr_ij (angular)
    const int32_t *freeze;  // MD: status word; the kernel does nothing once FREEZE_MASK is set
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
    // fused second half-kick (MD)
    float *v;               // [3][n] or null
    float half_dt_accel;    // dt/2 * ACCEL
    float dt;
    float inv_mass[MAXT];
    float mass[MAXT];
    const float *ref;       // [3][n] positions at the last build (rebuild prediction)
    const int32_t *freeze;  // MD: status word (see EfvArgs)
};

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

// Real solid-harmonic polynomials P_lm(u) for l = 1..4 on the unit sphere;
// with the weights N2 below, sum_m N2_lm P_lm(u) P_lm(v) = (2l+1)/(4 pi) P_l(u.v),
// so sum_m N2 A_lm^2 equals the complex sum of Eq. 4.
__device__ __forceinline__ void harmonics(float x, float y, float z, float P[LM]) {
    float x2 = x * x, y2 = y * y, z2 = z * z;
    P[0] = x; P[1] = y; P[2] = z;
    P[3] = x * y; P[4] = y * z; P[5] = x * z; P[6] = x2 - y2; P[7] = 3.0f * z2 - 1.0f;
    float a = 3.0f * x2 - y2, b = 5.0f * z2 - 1.0f, c = x2 - 3.0f * y2, d = x2 - y2;
    P[8] = y * a; P[9] = x * y * z; P[10] = y * b; P[11] = z * (5.0f * z2 - 3.0f);
    P[12] = x * b; P[13] = z * d; P[14] = x * c;
    float e = 7.0f * z2 - 1.0f, f = 7.0f * z2 - 3.0f;
    P[15] = x * y * d; P[16] = y * z * a; P[17] = x * y * e; P[18] = y * z * f;
    P[19] = (35.0f * z2 - 30.0f) * z2 + 3.0f; P[20] = x * z * f; P[21] = d * e;
    P[22] = x * z * c; P[23] = x2 * x2 - 6.0f * x2 * y2 + y2 * y2;
}

// V += sum_lm B_lm grad_u P_lm(u)   (polynomial gradients, unprojected)
__device__ __forceinline__ void harmonics_grad(float x, float y, float z, const float B[LM],
                                               float &vx, float &vy, float &vz) {
    float x2 = x * x, y2 = y * y, z2 = z * z;
    float xy = x * y, yz = y * z, xz = x * z, xyz = xy * z;
    vx += B[0]; vy += B[1]; vz += B[2];
    // l = 2
    vx += B[3] * y; vy += B[3] * x;
    vy += B[4] * z; vz += B[4] * y;
    vx += B[5] * z; vz += B[5] * x;
    vx += 2.0f * B[6] * x; vy -= 2.0f * B[6] * y;
    vz += 6.0f * B[7] * z;
    // l = 3
    float b51 = 5.0f * z2 - 1.0f, d = x2 - y2;
    vx += 6.0f * B[8] * xy; vy += 3.0f * B[8] * d;
    vx += B[9] * yz; vy += B[9] * xz; vz += B[9] * xy;
    vy += B[10] * b51; vz += 10.0f * B[10] * yz;
    vz += B[11] * (15.0f * z2 - 3.0f);
    vx += B[12] * b51; vz += 10.0f * B[12] * xz;
    vx += 2.0f * B[13] * xz; vy -= 2.0f * B[13] * yz; vz += B[13] * d;
    vx += 3.0f * B[14] * d; vy -= 6.0f * B[14] * xy;
    // l = 4
    float a3 = 3.0f * x2 - y2, c3 = x2 - 3.0f * y2;
    float e = 7.0f * z2 - 1.0f, f = 7.0f * z2 - 3.0f;
    vx += B[15] * y * a3; vy += B[15] * x * c3;
    vx += 6.0f * B[16] * xyz; vy += 3.0f * B[16] * z * d; vz += B[16] * y * a3;
    vx += B[17] * y * e; vy += B[17] * x * e; vz += 14.0f * B[17] * xyz;
    vy += B[18] * z * f; vz += B[18] * y * (21.0f * z2 - 3.0f);
    vz += B[19] * z * (140.0f * z2 - 60.0f);
    vx += B[20] * z * f; vz += B[20] * x * (21.0f * z2 - 3.0f);
    vx += 2.0f * B[21] * x * e; vy -= 2.0f * B[21] * y * e; vz += 14.0f * B[21] * z * d;
    vx += 3.0f * B[22] * z * d; vy -= 6.0f * B[22] * xyz; vz += B[22] * x * c3;
    vx += 4.0f * B[23] * x * c3; vy += 4.0f * B[23] * y * (y2 - 3.0f * x2);
}

__device__ __forceinline__ int lm_l(int lm) { return lm < 3 ? 1 : lm < 8 ? 2 : lm < 15 ? 3 : 4; }

// launchers (defined in the .hip files)
hipError_t launch_pack(int n, int T, const float *x, const float *y, const float *z, const uint8_t *type,
                       float4 *pos4, hipStream_t s);
hipError_t launch_efv_main(int T, const EfvArgs &a, size_t lds_bytes, hipStream_t s);
hipError_t launch_efv_gather(int T, bool virial, bool md, const GatherArgs &a, hipStream_t s);
hipError_t launch_reduce(const double *partial, int nblocks, double *E_tot, double *W_tot,
                         double *K_tot, double *E_slot, double *K_slot, double *counts,
                         const int32_t *status, double *info, hipStream_t s);
// rebuild prediction at the start of an MD call: maxima of |x + d - ref|,
// |d| and dt^2 |a| with d = dt (v + dt/2 a) the next drift, into the partials
struct PredictArgs {
    int n, T;
    const float *x, *y, *z, *v, *F, *ref;
    const uint8_t *type;
    float dt, half_dt_accel;
    float inv_mass[MAXT];
    double *partial;
};
hipError_t launch_predict(const PredictArgs &a, hipStream_t s);

struct NbArgs {
    int n, cap, cap_A;
    float box[3];
    int pbc[3];
    int nc[3], m[3];
    float inv_cs[3];
    float list2R[MAXT * MAXT], list2A[MAXT * MAXT];
    int T;
    const float *x, *y, *z;
    float *x_mut, *y_mut, *z_mut;  // same arrays, written only when wrap is set
    const uint8_t *type;
    float4 *pos4;
    int32_t *cell_id, *cell_count, *cell_start, *cell_cursor, *cell_list, *scan_tmp;
    uint32_t *nbr;
    int32_t *rev, *cnt;
    float *ref;
    int32_t *status;
    int ncell;
    int clear_status;  // 1: a fresh build resets the status word
    int wrap;          // 1: wrap periodic coordinates into [0, L) and write them back first
};
hipError_t launch_build(const NbArgs &a, hipStream_t s);
hipError_t launch_clear_status(int32_t *status, hipStream_t s);

struct KickDriftArgs {
    int n;
    float *x, *y, *z;
    float *v;               // [3][n]
    const float *F;         // [3][n]
    const uint8_t *type;
    float4 *pos4;
    float *ref;             // [3][n] positions at the last build
    float half_dt_accel;    // dt/2 * ACCEL
    float dt;
    float inv_mass[MAXT];
    float lam[3];           // affine scale factors of this step
    float box[3];           // box after the strain
    int pbc[3];
    int T;                  // number of types (type values are clamped below it)
    float half_skin2;       // (skin/2)^2
    int32_t *status;
};
hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t s);

}  // namespace nep
