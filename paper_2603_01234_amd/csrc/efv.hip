// NEP energy / force / virial kernels (paper Sec. II.A, Eqs. 2-8; forces from
// E = sum_i U_i; per-site virial of Eq. 15, total of Eq. 16).
//
// One thread per bead ("centre"), 256 beads per workgroup, XCD-aware tile map.
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
//               dU_i/dr_ij into a per-slot buffer, and their sum.
// k_efv_gather  F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji):
//               radial part of both terms from the pair geometry and the two
//               beads' beta vectors (no pair buffer); angular dU_j/dr_ji read
//               through the reverse index; per-site virial
//               W_i = sum_j r_ij (x) dU_j/dr_ji; fixed-order block sums of U,
//               W and (for MD) the kinetic energy; optional second half-kick.
// k_reduce      fixed-order FP64 reduction of the block sums.
#include "nep_internal.h"

namespace nep {

// N2_lm: squared normalisation of the real harmonics P_lm (l = 1..4)
#define PI_F 3.14159265358979f
__device__ constexpr float N2[LM] = {
    3.0f / (4 * PI_F), 3.0f / (4 * PI_F), 3.0f / (4 * PI_F),
    15.0f / (4 * PI_F), 15.0f / (4 * PI_F), 15.0f / (4 * PI_F), 15.0f / (16 * PI_F), 5.0f / (16 * PI_F),
    35.0f / (32 * PI_F), 105.0f / (4 * PI_F), 21.0f / (32 * PI_F), 7.0f / (16 * PI_F),
    21.0f / (32 * PI_F), 105.0f / (16 * PI_F), 35.0f / (32 * PI_F),
    315.0f / (16 * PI_F), 315.0f / (32 * PI_F), 45.0f / (16 * PI_F), 45.0f / (32 * PI_F),
    9.0f / (256 * PI_F), 45.0f / (32 * PI_F), 45.0f / (64 * PI_F), 315.0f / (32 * PI_F), 315.0f / (256 * PI_F)};

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

struct PairGeom {
    int j, tj;
    float dx, dy, dz, d2;
};

__device__ __forceinline__ PairGeom pair_geom(const float4 *__restrict__ pos4, uint32_t e,
                                              const float4 &pi, const float box[3]) {
    PairGeom g;
    int nx, ny, nz;
    decode(e, g.j, nx, ny, nz);
    float4 pj = pos4[g.j];
    g.dx = (pj.x + (float)nx * box[0]) - pi.x;
    g.dy = (pj.y + (float)ny * box[1]) - pi.y;
    g.dz = (pj.z + (float)nz * box[2]) - pi.z;
    g.d2 = g.dx * g.dx + g.dy * g.dy + g.dz * g.dz;
    g.tj = (int)pj.w;
    return g;
}

template <int NT>
__global__ __launch_bounds__(BLOCK) void k_efv_main(EfvArgs a) {
    extern __shared__ float smem[];
    const int H = a.H;
    const float *__restrict__ P;
    const float *__restrict__ TB;
    if constexpr (NT > 1) {
        // per-lane type indices: stage the network and coefficient tables in LDS
        int np = NT * H * (ND + 2) + 1;
        int nt = NT * NT * TAB_PER_PAIR;
        for (int k = threadIdx.x; k < np; k += BLOCK) smem[k] = a.params[k];
        for (int k = threadIdx.x; k < nt; k += BLOCK) smem[np + k] = a.tab[k];
        __syncthreads();
        P = smem;
        TB = smem + np;
    } else {
        // one type: every coefficient address is wave-uniform (scalar loads)
        P = a.params;
        TB = a.tab;
    }
    if (a.freeze && (a.freeze[0] & FREEZE_MASK)) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int i = tile * BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const int n = a.n;
    const float4 pi = a.pos4[i];
    const int ti = (NT == 1) ? 0 : (int)pi.w;
    const int cR = a.cnt[i];
    const int cA = a.cnt[n + i];

    float S[NT][KB];
    float A[NA][LM];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int k = 0; k < KB; ++k) S[t][k] = 0.0f;
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
        for (int l = 0; l < LM; ++l) A[q][l] = 0.0f;

    // ---------------- pass 1: descriptor sums ----------------
    for (int p = 0; p < cR; ++p) {
        PairGeom g = pair_geom(a.pos4, a.nbr[(size_t)p * n + i], pi, a.box);
        const int tj = (NT == 1) ? 0 : g.tj;
        const int tp = ti * NT + tj;
        if (g.d2 < a.cut.rcR2[tp]) {
            float r = sqrtf(g.d2);
            float t = r * a.cut.inv_rcR[tp];
            float hfc = 0.25f * (1.0f + cospif(t));
            float s1 = t - 1.0f;
            float T[KB];
            cheb_T(2.0f * s1 * s1 - 1.0f, T);
#pragma unroll
            for (int t2 = 0; t2 < NT; ++t2) {
                float w = (NT == 1 || tj == t2) ? hfc : 0.0f;
                S[t2][0] += w;
#pragma unroll
                for (int k = 1; k < KB; ++k) S[t2][k] += w * T[k];
            }
            if (p < cA && g.d2 < a.cut.rcA2[tp]) {
                float tA = r * a.cut.inv_rcA[tp];
                float hA = 0.25f * (1.0f + cospif(tA));
                float sA = tA - 1.0f;
                float TA[KB];
                cheb_T(2.0f * sA * sA - 1.0f, TA);
                const float *__restrict__ cAp = TB + tp * TAB_PER_PAIR + NR * KB;
                float gv[NA];
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    float G = cAp[q * KB];
#pragma unroll
                    for (int k = 1; k < KB; ++k) G += cAp[q * KB + k] * TA[k];
                    gv[q] = hA * G;
                }
                float ir = 1.0f / r;
                float Pl[LM];
                harmonics(g.dx * ir, g.dy * ir, g.dz * ir, Pl);
#pragma unroll
                for (int q = 0; q < NA; ++q)
#pragma unroll
                    for (int l = 0; l < LM; ++l) A[q][l] += gv[q] * Pl[l];
            }
        }
    }

    // ---------------- descriptor ----------------
    float qd[ND];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float *__restrict__ cRp = TB + (ti * NT + t) * TAB_PER_PAIR;
#pragma unroll
            for (int k = 0; k < KB; ++k) acc += cRp[q * KB + k] * S[t][k];
        }
        qd[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int l = 0; l < LM; ++l) s[lm_l(l) - 1] += N2[l] * A[q][l] * A[q][l];
#pragma unroll
        for (int L = 0; L < 4; ++L) qd[NR + L * NA + q] = s[L];
    }

    // ---------------- network (Eq. 2) and dU/dq ----------------
    const float *__restrict__ w0 = P + ti * H * ND;
    const float *__restrict__ b0 = P + NT * H * ND + ti * H;
    const float *__restrict__ w1 = P + NT * H * ND + NT * H + ti * H;
    const float b1 = P[NT * H * ND + 2 * NT * H];
    float U = -b1;
    float dq[ND];
#pragma unroll
    for (int v = 0; v < ND; ++v) dq[v] = 0.0f;
    for (int mu = 0; mu < H; ++mu) {
        float z = -b0[mu];
#pragma unroll
        for (int v = 0; v < ND; ++v) z += w0[mu * ND + v] * qd[v];
        float h = tanhf(z);
        float w1m = w1[mu];
        U += w1m * h;
        float s = w1m * (1.0f - h * h);
#pragma unroll
        for (int v = 0; v < ND; ++v) dq[v] += s * w0[mu * ND + v];
    }
    a.U[i] = U;

    // radial back-propagation coefficients per neighbour type
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const float *__restrict__ cRp = TB + (ti * NT + t) * TAB_PER_PAIR;
        float be[12];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < NR; ++q) acc += dq[q] * cRp[q * KB + k];
            be[k] = acc;
        }
        be[9] = be[10] = be[11] = 0.0f;
        float4 *dst = a.bvec + ((size_t)i * NT + t) * 3;
        dst[0] = make_float4(be[0], be[1], be[2], be[3]);
        dst[1] = make_float4(be[4], be[5], be[6], be[7]);
        dst[2] = make_float4(be[8], 0.0f, 0.0f, 0.0f);
    }

    // D_{n,lm} = dU/dq_nl * dq_nl/dA_{n,lm} = dU/dq_nl * 2 N2_lm A_{n,lm}
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
        for (int l = 0; l < LM; ++l) A[q][l] *= 2.0f * N2[l] * dq[NR + (lm_l(l) - 1) * NA + q];

    // ---------------- pass 2: angular pair partials ----------------
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    for (int p = 0; p < cA; ++p) {
        PairGeom g = pair_geom(a.pos4, a.nbr[(size_t)p * n + i], pi, a.box);
        const int tj = (NT == 1) ? 0 : g.tj;
        const int tp = ti * NT + tj;
        float ox = 0.0f, oy = 0.0f, oz = 0.0f;
        if (g.d2 < a.cut.rcA2[tp]) {
            float r = sqrtf(g.d2);
            float ir = 1.0f / r;
            float ux = g.dx * ir, uy = g.dy * ir, uz = g.dz * ir;
            float inv = a.cut.inv_rcA[tp];
            float tA = r * inv;
            float sp, cp;
            sincospif(tA, &sp, &cp);
            float hA = 0.25f * (1.0f + cp);
            float dhA = -0.25f * PI_F * sp * inv;
            float sA = tA - 1.0f;
            float xA = 2.0f * sA * sA - 1.0f;
            float xp = 4.0f * sA * inv;
            float TA[KB], UA[KB - 1];
            cheb_T(xA, TA);
            cheb_U(xA, UA);
            const float *__restrict__ cAp = TB + tp * TAB_PER_PAIR + NR * KB;
            const float *__restrict__ cAd = cAp + NA * KB;
            float gv[NA], gp[NA];
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                float G = cAp[q * KB], Gp = 0.0f;
#pragma unroll
                for (int k = 1; k < KB; ++k) {
                    G += cAp[q * KB + k] * TA[k];
                    Gp += cAd[q * (KB - 1) + k - 1] * UA[k - 1];
                }
                gv[q] = hA * G;
                gp[q] = dhA * G + hA * xp * Gp;
            }
            float Pl[LM], Bv[LM];
            harmonics(ux, uy, uz, Pl);
            float s = 0.0f;
#pragma unroll
            for (int l = 0; l < LM; ++l) {
                float B = 0.0f, Bp = 0.0f;
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    B += A[q][l] * gv[q];
                    Bp += A[q][l] * gp[q];
                }
                s += Bp * Pl[l];
                Bv[l] = B;
            }
            float vx = 0.0f, vy = 0.0f, vz = 0.0f;
            harmonics_grad(ux, uy, uz, Bv, vx, vy, vz);
            float uv = ux * vx + uy * vy + uz * vz;
            ox = s * ux + (vx - uv * ux) * ir;
            oy = s * uy + (vy - uv * uy) * ir;
            oz = s * uz + (vz - uv * uz) * ir;
        }
        a.angbuf[(size_t)p * n + i] = make_float4(ox, oy, oz, 0.0f);
        fx += ox;
        fy += oy;
        fz += oz;
    }
    a.fown[i] = make_float4(fx, fy, fz, 0.0f);
}

template <int NT, bool VIR, bool MD>
__global__ __launch_bounds__(BLOCK) void k_efv_gather(GatherArgs a) {
    __shared__ double red[NPART][BLOCK];
    __shared__ float redm[NMAX][BLOCK];
    if (MD && a.freeze && (a.freeze[0] & FREEZE_MASK)) return;  // uniform over the grid
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int i = tile * BLOCK + threadIdx.x;
    const int n = a.n;
    double acc[NPART];
    float mx[NMAX] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < NPART; ++c) acc[c] = 0.0;
    int nR_in = 0, nA_in = 0;  // pairs inside the interaction cutoffs (work accounting)
    if (i < n) {
        const float4 pi = a.pos4[i];
        const int ti = (NT == 1) ? 0 : (int)pi.w;
        const int cR = a.cnt[i];
        const int cA = a.cnt[n + i];
        float bi[NT][KB];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float4 *src = a.bvec + ((size_t)i * NT + t) * 3;
            float4 v0 = src[0], v1 = src[1], v2 = src[2];
            bi[t][0] = v0.x; bi[t][1] = v0.y; bi[t][2] = v0.z; bi[t][3] = v0.w;
            bi[t][4] = v1.x; bi[t][5] = v1.y; bi[t][6] = v1.z; bi[t][7] = v1.w;
            bi[t][8] = v2.x;
        }
        float4 fo = a.fown[i];
        float Fx = fo.x, Fy = fo.y, Fz = fo.z;
        float W[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) W[c] = 0.0f;
        for (int p = 0; p < cR; ++p) {
            PairGeom g = pair_geom(a.pos4, a.nbr[(size_t)p * n + i], pi, a.box);
            const int tj = (NT == 1) ? 0 : g.tj;
            const int tp = ti * NT + tj;
            if (g.d2 < a.cut.rcR2[tp]) {
                ++nR_in;
                nA_in += (p < cA && g.d2 < a.cut.rcA2[tp]) ? 1 : 0;
                float r = sqrtf(g.d2);
                float ir = 1.0f / r;
                float inv = a.cut.inv_rcR[tp];
                float t = r * inv;
                float sp, cp;
                sincospif(t, &sp, &cp);
                float hfc = 0.25f * (1.0f + cp);
                float dh = -0.25f * PI_F * sp * inv;
                float s1 = t - 1.0f;
                float x = 2.0f * s1 * s1 - 1.0f;
                float xp = 4.0f * s1 * inv;
                float T[KB], Uc[KB - 1];
                cheb_T(x, T);
                cheb_U(x, Uc);
                // own coefficients for the neighbour's type
                float b[KB];
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    float v = bi[0][k];
#pragma unroll
                    for (int t2 = 1; t2 < NT; ++t2) v = (tj == t2) ? bi[t2][k] : v;
                    b[k] = v;
                }
                // neighbour's coefficients for this bead's type
                const float4 *src = a.bvec + ((size_t)g.j * NT + ti) * 3;
                float4 v0 = src[0], v1 = src[1], v2 = src[2];
                float c[KB] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x};
                float Si = b[0], Sj = c[0], Di = 0.0f, Dj = 0.0f;
#pragma unroll
                for (int k = 1; k < KB; ++k) {
                    float dT = (float)k * Uc[k - 1];
                    Si += b[k] * T[k];
                    Sj += c[k] * T[k];
                    Di += b[k] * dT;
                    Dj += c[k] * dT;
                }
                float si = dh * Si + hfc * xp * Di;  // dU_i/dr along r_ij
                float sj = dh * Sj + hfc * xp * Dj;  // dU_j/dr along r_ji
                float ux = g.dx * ir, uy = g.dy * ir, uz = g.dz * ir;
                float st = si + sj;
                Fx += st * ux;
                Fy += st * uy;
                Fz += st * uz;
                if (VIR) {  // dU_j/dr_ji (radial part) = -sj u
                    float fx = -sj * ux, fy = -sj * uy, fz = -sj * uz;
                    W[0] += g.dx * fx; W[1] += g.dx * fy; W[2] += g.dx * fz;
                    W[3] += g.dy * fx; W[4] += g.dy * fy; W[5] += g.dy * fz;
                    W[6] += g.dz * fx; W[7] += g.dz * fy; W[8] += g.dz * fz;
                }
            }
            if (p < cA) {
                int q = a.rev[(size_t)p * n + i];
                if (q >= 0) {
                    float4 fj = a.angbuf[q];  // dU_j/dr_ji, angular part
                    Fx -= fj.x;
                    Fy -= fj.y;
                    Fz -= fj.z;
                    if (VIR) {
                        W[0] += g.dx * fj.x; W[1] += g.dx * fj.y; W[2] += g.dx * fj.z;
                        W[3] += g.dy * fj.x; W[4] += g.dy * fj.y; W[5] += g.dy * fj.z;
                        W[6] += g.dz * fj.x; W[7] += g.dz * fj.y; W[8] += g.dz * fj.z;
                    }
                }
            }
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
        if (MD) {
            float k = a.half_dt_accel * a.inv_mass[ti];
            float vx = a.v[i] + k * Fx;
            float vy = a.v[n + i] + k * Fy;
            float vz = a.v[2 * n + i] + k * Fz;
            a.v[i] = vx;
            a.v[n + i] = vy;
            a.v[2 * n + i] = vz;
            acc[10] = 0.5 * (double)a.mass[ti] * ((double)vx * vx + (double)vy * vy + (double)vz * vz) /
                      (double)ACCEL;
            // next drift d = dt (v + dt/2 a): displacement from the build
            // reference after it, |d|, and dt^2 |a| (rebuild prediction)
            float ddx = a.dt * (vx + k * Fx), ddy = a.dt * (vy + k * Fy), ddz = a.dt * (vz + k * Fz);
            float px = pi.x + ddx - a.ref[i], py = pi.y + ddy - a.ref[n + i], pz = pi.z + ddz - a.ref[2 * n + i];
            mx[0] = px * px + py * py + pz * pz;
            mx[1] = ddx * ddx + ddy * ddy + ddz * ddz;
            mx[2] = 2.0f * a.dt * k * sqrtf(Fx * Fx + Fy * Fy + Fz * Fz);
        }
    }
    if (MD) {
#pragma unroll
        for (int c = 0; c < NMAX; ++c) redm[c][threadIdx.x] = mx[c];
    }
    // fixed-order block reduction
#pragma unroll
    for (int c = 0; c < NPART; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < NPART; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
            if (MD)
#pragma unroll
                for (int c = 0; c < NMAX; ++c) redm[c][threadIdx.x] = fmaxf(redm[c][threadIdx.x], redm[c][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < NPART) a.partial[(size_t)tile * 16 + threadIdx.x] = red[threadIdx.x][0];
    if (threadIdx.x < NMAX) a.partial[(size_t)tile * 16 + NPART + threadIdx.x] = MD ? (double)redm[threadIdx.x][0] : 0.0;
}

__global__ __launch_bounds__(BLOCK) void k_predict(PredictArgs a) {
    __shared__ double red[NPART][BLOCK];
    __shared__ float redm[NMAX][BLOCK];
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    const int n = a.n;
    float mx[NMAX] = {0.0f, 0.0f, 0.0f};
    if (i < n) {
        int t = min((int)a.type[i], a.T - 1);
        float k = a.half_dt_accel * a.inv_mass[t];
        float Fx = a.F[i], Fy = a.F[n + i], Fz = a.F[2 * n + i];
        float ddx = a.dt * (a.v[i] + k * Fx), ddy = a.dt * (a.v[n + i] + k * Fy), ddz = a.dt * (a.v[2 * n + i] + k * Fz);
        float px = a.x[i] + ddx - a.ref[i], py = a.y[i] + ddy - a.ref[n + i], pz = a.z[i] + ddz - a.ref[2 * n + i];
        mx[0] = px * px + py * py + pz * pz;
        mx[1] = ddx * ddx + ddy * ddy + ddz * ddz;
        mx[2] = 2.0f * a.dt * k * sqrtf(Fx * Fx + Fy * Fy + Fz * Fz);
    }
#pragma unroll
    for (int c = 0; c < NPART; ++c) red[c][threadIdx.x] = 0.0;
#pragma unroll
    for (int c = 0; c < NMAX; ++c) redm[c][threadIdx.x] = mx[c];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int c = 0; c < NMAX; ++c) redm[c][threadIdx.x] = fmaxf(redm[c][threadIdx.x], redm[c][threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x < NPART) a.partial[(size_t)blockIdx.x * 16 + threadIdx.x] = 0.0;
    if (threadIdx.x < NMAX) a.partial[(size_t)blockIdx.x * 16 + NPART + threadIdx.x] = (double)redm[threadIdx.x][0];
}

hipError_t launch_predict(const PredictArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict, dim3((a.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// Fixed-order FP64 reduction of the block partials.  In MD mode (status and
// info given) it also takes the maxima of the rebuild prediction and writes
// one info record straight into pinned host memory:
//   info = {E, K, max|x + d - ref|, max|d|, max dt^2|a|, status[0..2]}
// Once the status carries a freeze flag the energy outputs are left alone.
__global__ void k_reduce(const double *__restrict__ partial, int nblocks, double *E_tot,
                         double *W_tot, double *K_tot, double *E_slot, double *K_slot, double *counts,
                         const int32_t *status, double *info) {
    __shared__ double red[NPART + NMAX][BLOCK];
    double acc[NPART + NMAX];
#pragma unroll
    for (int c = 0; c < NPART + NMAX; ++c) acc[c] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += BLOCK) {
#pragma unroll
        for (int c = 0; c < NPART; ++c) acc[c] += partial[(size_t)b * 16 + c];
#pragma unroll
        for (int c = NPART; c < NPART + NMAX; ++c) acc[c] = fmax(acc[c], partial[(size_t)b * 16 + c]);
    }
#pragma unroll
    for (int c = 0; c < NPART + NMAX; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < NPART; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
#pragma unroll
            for (int c = NPART; c < NPART + NMAX; ++c) red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + s]);
        }
        __syncthreads();
    }
    const int st0 = status ? status[0] : 0;
    if (threadIdx.x == 0 && info) {
        info[0] = red[0][0];
        info[1] = red[10][0];
        info[2] = sqrt(red[NPART][0]);
        info[3] = sqrt(red[NPART + 1][0]);
        info[4] = red[NPART + 2][0];
        info[5] = (double)st0;
        info[6] = (double)status[1];
        info[7] = (double)status[2];
    }
    if (st0 & FREEZE_MASK) return;
    if (threadIdx.x == 0) {
        if (E_tot) *E_tot = red[0][0];
        if (E_slot) *E_slot = red[0][0];
        if (K_tot) *K_tot = red[10][0];
        if (K_slot) *K_slot = red[10][0];
        if (counts) {
            counts[0] += red[11][0];
            counts[1] += red[12][0];
        }
    }
    if (W_tot && threadIdx.x < 9) W_tot[threadIdx.x] = red[1 + threadIdx.x][0];
}

hipError_t launch_reduce(const double *partial, int nblocks, double *E_tot, double *W_tot,
                         double *K_tot, double *E_slot, double *K_slot, double *counts,
                         const int32_t *status, double *info, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(BLOCK), 0, s, partial, nblocks, E_tot, W_tot, K_tot,
                       E_slot, K_slot, counts, status, info);
    return hipGetLastError();
}

template <int NT>
static hipError_t main_t(const EfvArgs &a, size_t lds, hipStream_t s) {
    int nb = (a.n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_efv_main<NT>, dim3(nb), dim3(BLOCK), NT > 1 ? lds : 0, s, a);
    return hipGetLastError();
}

hipError_t launch_efv_main(int T, const EfvArgs &a, size_t lds, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (T) {
        case 1: return main_t<1>(a, lds, s);
        case 2: return main_t<2>(a, lds, s);
        case 3: return main_t<3>(a, lds, s);
        case 4: return main_t<4>(a, lds, s);
    }
    return hipErrorInvalidValue;
}

template <int NT, bool VIR, bool MD>
static hipError_t gather_t(const GatherArgs &a, hipStream_t s) {
    int nb = (a.n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL((k_efv_gather<NT, VIR, MD>), dim3(nb), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int NT>
static hipError_t gather_nt(bool vir, bool md, const GatherArgs &a, hipStream_t s) {
    if (vir) return md ? gather_t<NT, true, true>(a, s) : gather_t<NT, true, false>(a, s);
    return md ? gather_t<NT, false, true>(a, s) : gather_t<NT, false, false>(a, s);
}

hipError_t launch_efv_gather(int T, bool vir, bool md, const GatherArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (T) {
        case 1: return gather_nt<1>(vir, md, a, s);
        case 2: return gather_nt<2>(vir, md, a, s);
        case 3: return gather_nt<3>(vir, md, a, s);
        case 4: return gather_nt<4>(vir, md, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace nep
