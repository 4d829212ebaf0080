// Device-side building blocks of the NEP energy / force / virial evaluation
// (Sec. II.A, Eqs. 2-8, forces from E = sum_i U_i, per-site virial Eq. 15),
// shared by the single-system kernels and the batched fitness kernel.
#pragma once
#include <type_traits>

#include "nep_internal.h"

namespace nep {

// N2_lm: squared normalisation of the real harmonics P_lm (l = 1..4)
#define PI_F 3.14159265358979f
static __device__ constexpr float N2[LM] = {
    3.0f / (4 * PI_F), 3.0f / (4 * PI_F), 3.0f / (4 * PI_F),
    15.0f / (4 * PI_F), 15.0f / (4 * PI_F), 15.0f / (4 * PI_F), 15.0f / (16 * PI_F), 5.0f / (16 * PI_F),
    35.0f / (32 * PI_F), 105.0f / (4 * PI_F), 21.0f / (32 * PI_F), 7.0f / (16 * PI_F),
    21.0f / (32 * PI_F), 105.0f / (16 * PI_F), 35.0f / (32 * PI_F),
    315.0f / (16 * PI_F), 315.0f / (32 * PI_F), 45.0f / (16 * PI_F), 45.0f / (32 * PI_F),
    9.0f / (256 * PI_F), 45.0f / (32 * PI_F), 45.0f / (64 * PI_F), 315.0f / (32 * PI_F), 315.0f / (256 * PI_F)};

struct PairGeom {
    int j, tj;
    float dx, dy, dz, d2;
};


__device__ __forceinline__ PairGeom geom_of(uint32_t e, const float4 &pj, const float4 &pi,
                                            const float box[3]) {
    PairGeom g;
    int nx, ny, nz;
    decode(e, g.j, nx, ny, nz);
    g.dx = (pj.x + (float)nx * box[0]) - pi.x;
    g.dy = (pj.y + (float)ny * box[1]) - pi.y;
    g.dz = (pj.z + (float)nz * box[2]) - pi.z;
    g.d2 = g.dx * g.dx + g.dy * g.dy + g.dz * g.dz;
    g.tj = (int)pj.w;
    return g;
}

// Neighbour stream of one row with software prefetch: the entry two slots
// ahead and the position one slot ahead are in flight while the current pair
// is processed.
struct RowStream {
    const uint32_t *__restrict__ nbr;
    const float4 *__restrict__ pos4;
    int n, i, cnt, step;
    uint32_t e_cur, e_nxt;
    float4 p_cur;
    // slots p0, p0 + step, p0 + 2 step, ... of row i (c entries in the row)
    __device__ __forceinline__ void start(const uint32_t *nb, const float4 *pp, int n_, int i_, int c,
                                          int p0 = 0, int step_ = 1) {
        nbr = nb;
        pos4 = pp;
        n = n_;
        i = i_;
        cnt = c;
        step = step_;
        e_cur = p0 < c ? nbr[(size_t)p0 * n + i] : 0u;
        e_nxt = p0 < c ? nbr[(size_t)min(p0 + step, c - 1) * n + i] : 0u;
        p_cur = p0 < c ? pos4[e_cur & J_MASK] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    // The pair geometry of slot p (called only for slots p < cnt), then the
    // look-ahead loads.  These are unconditional (past the end they read the
    // row's last entry again): a conditional load makes the compiler wait for
    // every load in flight at the join, which would take away the look-ahead.
    __device__ __forceinline__ PairGeom next_geom(int p, const float4 &pi, const float box[3]) {
        const PairGeom g = geom_of(e_cur, p_cur, pi, box);
        e_cur = e_nxt;
        e_nxt = nbr[(size_t)min(p + 2 * step, cnt - 1) * n + i];
        p_cur = pos4[e_cur & J_MASK];
        return g;
    }
};

// Slots 0, 1, ... of row i (c entries) in S interleaved sets (slot p belongs
// to set p mod S), each with its own registers: a set's position is loaded S
// slots ahead and its entry 2 S slots ahead.  The rounds of S slots are
// unrolled by two, the entries of even rounds in X and of odd rounds in Y, so
// each load writes the register whose value was just used (an entry once its
// pair is decoded and its successor's position issued) and the loop carries
// no register copies: a copy at the back edge would wait for the load it
// copies and take the look-ahead away.  The loads are unconditional and
// clamped to the row's last entry; body(p, g) runs for slots p < c, in slot
// order.
template <int S, class Body>
__device__ __forceinline__ void for_each_slot(const uint32_t *__restrict__ nbr, const float4 *__restrict__ pos4,
                                              int n, int i, int c, const float4 &pi, const float box[3],
                                              Body &&body) {
    if (c <= 0) return;
    const int last = c - 1;
    auto entry = [&](int p) { return nbr[(size_t)min(p, last) * n + i]; };
    uint32_t X[S], Y[S];
    float4 P[S];
#pragma unroll
    for (int k = 0; k < S; ++k) X[k] = entry(k);
#pragma unroll
    for (int k = 0; k < S; ++k) {
        P[k] = pos4[X[k] & J_MASK];
        Y[k] = entry(S + k);
    }
    for (int p = 0; p < c; p += 2 * S) {
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const PairGeom g = geom_of(X[k], P[k], pi, box);
            P[k] = pos4[Y[k] & J_MASK];
            X[k] = entry(p + 2 * S + k);
            if (k == 0 || p + k < c) body(p + k, g);
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const PairGeom g = geom_of(Y[k], P[k], pi, box);
            P[k] = pos4[X[k] & J_MASK];
            Y[k] = entry(p + 3 * S + k);
            if (p + S + k < c) body(p + S + k, g);
        }
    }
}

// Tables read through the constant address space: with wave-uniform addresses
// (one type) these become scalar loads whose values feed the FMAs as SGPR
// operands, so the weights never occupy vector registers.
typedef const __attribute__((address_space(4))) float *const_fp;

// Loads from the constant address space count as invariant, so the compiler
// may issue all of them long before use, whatever the memory barriers say,
// and then spill the scalar registers that hold them.  Passing a row's
// address through an empty asm makes it unknown until that row is reached,
// so each row of weights is loaded just before its use.
// a wave-uniform pointer moved into scalar registers
__device__ __forceinline__ const float *uniform_ptr(const float *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const float *)(((uint64_t)hi << 32) | lo);
}

// The address must be wave-uniform (it is for every table read here); it is
// moved to scalar registers first in case it was loaded into vector ones.
__device__ __forceinline__ const_fp opaque(const_fp p) {
    uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    v = ((uint64_t)hi << 32) | lo;
    asm volatile("" : "+s"(v));
    return (const_fp)v;
}

template <int NT>
using table_ptr = typename std::conditional<NT == 1, const_fp, const float *>::type;

// Descriptor from the pair sums, the network (Eq. 2) with its gradient, the
// radial back-propagation coefficients (written to bvec_out), and the angular
// gradient folded into A (D_{n,lm} = dU/dq_nl 2 N2_lm A_{n,lm}).  ti is
// wave-uniform, so every table read is a scalar load.
template <int NT, int HP>
__device__ __forceinline__ void network(const int ti, const const_fp TB, const const_fp AN,
                                        const float S[NT][KB], float A[NA][LM], float *U_out,
                                        float4 *bvec_out) {
    asm volatile("" ::: "memory");
    // ---------------- descriptor and network (Eq. 2), nu-outer ----------------
    const const_fp an = AN + ti * (ND + 2) * HP;  // w0T[ND][HP], b0[HP], w1[HP]
    float z[HP];
#pragma unroll
    for (int m = 0; m < HP; ++m) z[m] = -an[ND * HP + m];
    // one row of weights (and of pair coefficients) in flight at a time
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        float qv = 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const const_fp cRq = opaque(TB + (ti * NT + t) * TAB_PER_PAIR + q * KB);
#pragma unroll
            for (int k = 0; k < KB; ++k) qv += cRq[k] * S[t][k];
        }
        const const_fp w = opaque(an + q * HP);
#pragma unroll
        for (int m = 0; m < HP; ++m) z[m] += w[m] * qv;
    }
#pragma unroll
    for (int L = 1; L <= 4; ++L)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            float qv = 0.0f;
#pragma unroll
            for (int l = 0; l < LM; ++l)
                if (lm_l(l) == L) qv += N2[l] * A[q][l] * A[q][l];
            const int nu = NR + (L - 1) * NA + q;
            const const_fp w = opaque(an + nu * HP);
#pragma unroll
            for (int m = 0; m < HP; ++m) z[m] += w[m] * qv;
        }
    float U = -AN[NT * (ND + 2) * HP];
    const const_fp w1 = opaque(an + (ND + 1) * HP);
#pragma unroll
    for (int m = 0; m < HP; ++m) {
        const float h = tanh_nobranch(z[m]);
        const float w1m = w1[m];
        U += w1m * h;
        z[m] = w1m * (1.0f - h * h);  // dU/dz_m
    }
    *U_out = U;

    // dU/dq, nu-outer: radial part kept, angular part folded into
    // D_{n,lm} = dU/dq_nl * 2 N2_lm A_{n,lm}  (in place of A); the weights
    // are loaded again row by row rather than kept from the forward pass
    float dr[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const const_fp w = opaque(an + q * HP);
        float acc = 0.0f;
#pragma unroll
        for (int m = 0; m < HP; ++m) acc += z[m] * w[m];
        // computed here, next to its weights: left free, the arithmetic is
        // sunk towards its use and the loaded weights stay live (and spill)
        asm volatile("" : "+v"(acc));
        dr[q] = acc;
    }
#pragma unroll
    for (int L = 1; L <= 4; ++L)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int nu = NR + (L - 1) * NA + q;
            const const_fp w = opaque(an + nu * HP);
            float acc = 0.0f;
#pragma unroll
            for (int m = 0; m < HP; ++m) acc += z[m] * w[m];
            asm volatile("" : "+v"(acc));
#pragma unroll
            for (int l = 0; l < LM; ++l)
                if (lm_l(l) == L) A[q][l] *= 2.0f * N2[l] * acc;
        }
    asm volatile("" ::: "memory");

    // radial back-propagation coefficients per neighbour type:
    //   beta_k = sum_n dU/dq_n c'_nk   (k = 0 uses c'_n0 = c_n0 + sum_k c_nk)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        float be[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) be[k] = 0.0f;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const const_fp cRq = opaque(TB + (ti * NT + t) * TAB_PER_PAIR + q * KB);
#pragma unroll
            for (int k = 0; k < KB; ++k) be[k] += dr[q] * cRq[k];
        }
        float4 *dst = bvec_out + (size_t)t * 3;
        dst[0] = make_float4(be[0], be[1], be[2], be[3]);
        dst[1] = make_float4(be[4], be[5], be[6], be[7]);
        dst[2] = make_float4(be[8], 0.0f, 0.0f, 0.0f);
    }

}

// ---------------- the network on the matrix cores ----------------
// The same contraction as network() for one bead type, over the 64 beads of a
// wavefront: Z = Q W0 - b0 (beads x ND times ND x HP) and dU/dq = DZ W0^T
// (beads x HP times HP x ND) as FP32 16x16x4 MFMAs.  The lanes hold one bead
// each, the MFMA operands a 16 x 4 tile of beads x k (lane l: row l % 16,
// column l / 16) and a 4 x 16 tile of k x columns (lane l: row l / 16, column
// l % 16), the results a 16 x 16 tile (lane l: rows 4 (l / 16) .. + 3, column
// l % 16); the layouts are exchanged through LDS.
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int MF_WROWS = 48;  // W0 rows staged: ND = 37 padded to three 16-row tiles (zeros)
// LDS row stride (floats) of a wavefront's bead tile: the descriptor rows,
// then in the same 16-row blocks the hidden-unit gradients [HP][16] and the
// descriptor gradients [48][16]
template <int HP>
__host__ __device__ constexpr int mf_stride() { return HP > 48 ? HP + 4 : 52; }
template <int HP>
__host__ __device__ constexpr int mf_lds_floats(int waves) {
    return MF_WROWS * (HP + 1) + waves * (64 * mf_stride<HP>() + 64);
}

// stage W0 (one type) as [48][HP + 1] (the pad column spreads the columns of
// the backward operand over the banks); rows past ND are zero
template <int HP>
__device__ __forceinline__ void mf_stage_w0(const float *__restrict__ ann, float *w0s) {
    for (int e = threadIdx.x; e < MF_WROWS * HP; e += blockDim.x) {
        const int r = e / HP, c = e % HP;
        w0s[r * (HP + 1) + c] = r < ND ? ann[r * HP + c] : 0.0f;
    }
}

template <int HP>
__device__ __forceinline__ void network_mfma(const const_fp TB, const const_fp AN, const float S[1][KB],
                                             float A[NA][LM], float *U_out, float4 *bvec_out, bool take,
                                             const float *w0s, float *wl) {
    constexpr int QS = mf_stride<HP>();
    constexpr int NT16 = HP / 16;
    const int lane = __lane_id();
    const int r16 = lane & 15, g4 = lane >> 4;
    float *us = wl + 64 * QS;  // per-bead sums of w1 h
    asm volatile("" ::: "memory");
    // descriptor of this lane's bead into its row (q_37..39 = 0 pad the last k step)
    {
        float *row = wl + lane * QS;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const const_fp cRq = opaque(TB + q * KB);
            float qv = 0.0f;
#pragma unroll
            for (int k = 0; k < KB; ++k) qv += cRq[k] * S[0][k];
            row[q] = qv;
        }
#pragma unroll
        for (int L = 1; L <= 4; ++L)
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                float qv = 0.0f;
#pragma unroll
                for (int l = 0; l < LM; ++l)
                    if (lm_l(l) == L) qv += N2[l] * A[q][l] * A[q][l];
                row[NR + (L - 1) * NA + q] = qv;
            }
        row[ND] = row[ND + 1] = row[ND + 2] = 0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // forward, 16 beads at a time; the tile's hidden-unit gradients replace its
    // descriptor rows once they are read
    float b0c[NT16], w1c[NT16];
#pragma unroll
    for (int nt = 0; nt < NT16; ++nt) {
        b0c[nt] = AN[ND * HP + 16 * nt + r16];
        w1c[nt] = AN[(ND + 1) * HP + 16 * nt + r16];
    }
#pragma unroll 1
    for (int mt = 0; mt < 4; ++mt) {
        float *tile = wl + mt * 16 * QS;
        v4f C[NT16];
#pragma unroll
        for (int nt = 0; nt < NT16; ++nt) C[nt] = v4f{-b0c[nt], -b0c[nt], -b0c[nt], -b0c[nt]};
#pragma unroll
        for (int ks = 0; ks < 10; ++ks) {
            const float av = tile[r16 * QS + 4 * ks + g4];
#pragma unroll
            for (int nt = 0; nt < NT16; ++nt)
                C[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, w0s[(4 * ks + g4) * (HP + 1) + 16 * nt + r16],
                                                             C[nt], 0, 0, 0);
        }
        float u[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int nt = 0; nt < NT16; ++nt) {
            float dz[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float h = tanh_nobranch(C[nt][v]);
                u[v] += w1c[nt] * h;
                dz[v] = w1c[nt] * (1.0f - h * h);
            }
            // [m][16 beads] of the tile
            *reinterpret_cast<float4 *>(tile + (16 * nt + r16) * 16 + 4 * g4) = make_float4(dz[0], dz[1], dz[2], dz[3]);
        }
        // sum over the hidden units: the 16 lanes of a column group hold them
#pragma unroll
        for (int o = 1; o < 16; o <<= 1)
#pragma unroll
            for (int v = 0; v < 4; ++v) u[v] += __shfl_xor(u[v], o, 16);
        if (r16 == 0) *reinterpret_cast<float4 *>(us + 16 * mt + 4 * g4) = make_float4(u[0], u[1], u[2], u[3]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // backward: dU/dq = DZ W0^T, 16 beads at a time, written back as [48][16 beads]
#pragma unroll 1
    for (int mt = 0; mt < 4; ++mt) {
        float *tile = wl + mt * 16 * QS;
        v4f D[3] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int ks = 0; ks < HP / 4; ++ks) {
            const float av = tile[(4 * ks + g4) * 16 + r16];
#pragma unroll
            for (int nt = 0; nt < 3; ++nt)
                D[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, w0s[(16 * nt + r16) * (HP + 1) + 4 * ks + g4], D[nt],
                                                             0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int nt = 0; nt < 3; ++nt)
            *reinterpret_cast<float4 *>(tile + (16 * nt + r16) * 16 + 4 * g4) =
                make_float4(D[nt][0], D[nt][1], D[nt][2], D[nt][3]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // back to one bead per lane: dU/dq of this lane's bead
    const float *dq = wl + (lane >> 4) * 16 * QS + (lane & 15);  // dq[nu] = dq[nu * 16]
    if (take) *U_out = us[lane] - AN[ND * HP + 2 * HP];
    float dr[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) dr[q] = dq[q * 16];
#pragma unroll
    for (int L = 1; L <= 4; ++L)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const float g = dq[(NR + (L - 1) * NA + q) * 16];
#pragma unroll
            for (int l = 0; l < LM; ++l)
                if (lm_l(l) == L) A[q][l] *= 2.0f * N2[l] * g;
        }
    asm volatile("" ::: "memory");
    // radial back-propagation coefficients
    float be[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) be[k] = 0.0f;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const const_fp cRq = opaque(TB + q * KB);
#pragma unroll
        for (int k = 0; k < KB; ++k) be[k] += dr[q] * cRq[k];
    }
    if (take) {
        bvec_out[0] = make_float4(be[0], be[1], be[2], be[3]);
        bvec_out[1] = make_float4(be[4], be[5], be[6], be[7]);
        bvec_out[2] = make_float4(be[8], 0.0f, 0.0f, 0.0f);
    }
}

// One centre bead of the fused kernel: both passes over its list and the
// network.  The cutoff tables are passed apart from the arguments so that they
// stay in kernel-argument memory (they are indexed by the lane's type pair).  Called with the lanes of beads that exist; for several types the
// lanes of one wave take part in the waterfall over centre types together.
// MF: the network on the matrix cores (one type; every lane of the wave calls
// with its bead, a lane past the system's end with valid = false, which keeps
// it out of the passes and the outputs); w0s and wl: the staged W0 and the
// wavefront's scratch in LDS.
template <int NT, int HP, bool MF = false>
__device__ __forceinline__ void main_bead(const EfvArgs &a, const Cut &cut, const table_ptr<NT> TB,
                                          const int i, const bool valid = true, const float *w0s = nullptr,
                                          float *wl = nullptr) {
    const int n = a.n;
    const float4 pi = a.pos4[i];
    const int ti = (NT == 1) ? 0 : (int)pi.w;
    const int cR = valid ? a.cnt[i] : 0;
    const int cA = valid ? a.cnt[n + i] : 0;

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
    // (three-set stream, rounds unrolled by two: the radial-only slots are
    // short, so one slot of look-ahead does not cover the position loads;
    // before the unrolling took the back-edge copies away, 2, 3, 4, 5 and 6
    // sets measured 373, 367, 364, 362 and 364 us on a hot 216,000-bead
    // system, and with it three and five sets are within 1% of each other)
    auto pass1 = [&](const int p, const PairGeom &g) {
        const int tj = (NT == 1) ? 0 : g.tj;
        const int tp = ti * NT + tj;
        if (g.d2 < cut.rcR2[tp]) {
            const float ir = __builtin_amdgcn_rsqf(g.d2);
            const float r = g.d2 * ir;
            const float t = r * cut.inv_rcR[tp];
            const float hfc = 0.25f * (1.0f + cos_pi(t));
            const float s1 = t - 1.0f;
            float T[KB];
            cheb_T(2.0f * s1 * s1 - 1.0f, T);
#pragma unroll
            for (int t2 = 0; t2 < NT; ++t2) {
                const float w = (NT == 1 || tj == t2) ? hfc : 0.0f;
                S[t2][0] += w;
#pragma unroll
                for (int k = 1; k < KB; ++k) S[t2][k] += w * T[k];
            }
            if (p < cA && g.d2 < cut.rcA2[tp]) {
                const float tA = r * cut.inv_rcA[tp];
                const float hA = 0.25f * (1.0f + cos_pi(tA));
                const float sA = tA - 1.0f;
                float TA[KB];
                cheb_T(2.0f * sA * sA - 1.0f, TA);
                const table_ptr<NT> cAp = TB + tp * TAB_PER_PAIR + NR * KB;
                float gv[NA];
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    float G = cAp[q * KB];
#pragma unroll
                    for (int k = 1; k < KB; ++k) G += cAp[q * KB + k] * TA[k];
                    gv[q] = hA * G;
                }
                accumulate_harmonics(g.dx * ir, g.dy * ir, g.dz * ir, gv, A);
            }
        }
    };
    for_each_slot<3>(a.nbr, a.pos4, n, i, cR, pi, a.box, pass1);

    // ---------------- descriptor, network (Eq. 2), back-propagation ----------------
    // evaluated with a wave-uniform centre type so the weights are scalar loads;
    // several types in one wave are handled one after the other
    if constexpr (MF) {
        static_assert(NT == 1, "the matrix-core network takes one bead type");
        network_mfma<HP>((const_fp)a.tab, (const_fp)a.ann, S, A, a.U + i, a.bvec + (size_t)i * 3, valid, w0s, wl);
    } else if constexpr (NT == 1) {
        network<NT, HP>(0, (const_fp)a.tab, (const_fp)a.ann, S, A, a.U + i, a.bvec + (size_t)i * NT * 3);
    } else {
        // the lane test goes through the ballot bit, not ti == tu, so the
        // compiler cannot substitute the per-lane ti into the table address
        uint64_t todo = __ballot(1);
        const int lane = __lane_id();
        while (todo) {
            const int lead = __ffsll((unsigned long long)todo) - 1;
            const int tu = __builtin_amdgcn_readfirstlane(__shfl(ti, lead));
            const uint64_t mine = __ballot(ti == tu);
            if ((mine >> lane) & 1ull)
                network<NT, HP>(tu, (const_fp)a.tab, (const_fp)a.ann, S, A, a.U + i,
                                a.bvec + (size_t)i * NT * 3);
            todo &= ~mine;
        }
    }
    asm volatile("" ::: "memory");
    // ---------------- pass 2: angular pair partials ----------------
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    RowStream rs;
    rs.start(a.nbr, a.pos4, n, i, cA);
    for (int p = 0; p < cA; ++p) {
        // the reverse slot is read before the look-ahead loads are issued, so
        // the wait for it at the store leaves them in flight
        const int r = a.rev[(size_t)p * n + i];
        const PairGeom g = rs.next_geom(p, pi, a.box);
        const int tj = (NT == 1) ? 0 : g.tj;
        const int tp = ti * NT + tj;
        float ox = 0.0f, oy = 0.0f, oz = 0.0f;
        if (g.d2 < cut.rcA2[tp]) {
            const float ir = __builtin_amdgcn_rsqf(g.d2);
            const float r = g.d2 * ir;
            const float ux = g.dx * ir, uy = g.dy * ir, uz = g.dz * ir;
            const float inv = cut.inv_rcA[tp];
            const float tA = r * inv;
            const float sp = sin_pi(tA), cp = cos_pi(tA);
            const float hA = 0.25f * (1.0f + cp);
            const float dhA = -0.25f * PI_F * sp * inv;
            const float sA = tA - 1.0f;
            const float xA = 2.0f * sA * sA - 1.0f;
            const float xp = 4.0f * sA * inv;
            float TA[KB], UA[KB - 1];
            cheb_T(xA, TA);
            cheb_U(xA, UA);
            const table_ptr<NT> cAp = TB + tp * TAB_PER_PAIR + NR * KB;
            // T_k' = k U_{k-1}: the derivative takes the same coefficients
            float dT[KB];
#pragma unroll
            for (int k = 1; k < KB; ++k) dT[k] = (float)k * UA[k - 1];
            float gv[NA], gp[NA];
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                float G = cAp[q * KB], Gp = 0.0f;
#pragma unroll
                for (int k = 1; k < KB; ++k) {
                    G += cAp[q * KB + k] * TA[k];
                    Gp += cAp[q * KB + k] * dT[k];
                }
                gv[q] = hA * G;
                gp[q] = dhA * G + hA * xp * Gp;
            }
            float s = 0.0f, vx = 0.0f, vy = 0.0f, vz = 0.0f;
            force_harmonics(ux, uy, uz, A, gv, gp, s, vx, vy, vz);
            const float uv = ux * vx + uy * vy + uz * vz;
            ox = s * ux + (vx - uv * ux) * ir;
            oy = s * uy + (vy - uv * uy) * ir;
            oz = s * uz + (vz - uv * uz) * ir;
        }
        // deliver dU_i/dr_ij to the slot where j lists i, for every pair that
        // j may find inside r_c^A (zero past it); a slot whose mirror does not
        // exist (rounding at the list edge) is zeroed by its owner
        if (g.d2 < cut.rcA2w[tp]) {
            if (r >= 0)
                a.angbuf[r] = make_float4(ox, oy, oz, 0.0f);
            else
                a.angbuf[(size_t)p * n + i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        fx += ox;
        fy += oy;
        fz += oz;
    }
    if (valid) a.fown[i] = make_float4(fx, fy, fz, 0.0f);
}

// Force and per-site virial of one bead from the pair terms of both beads of
// every pair (radial from the two beta vectors, angular from the reverse slot).
// Also counts the pairs inside the interaction cutoffs.
// Slots p0, p0 + step, ... of the row; the bead's own angular sum (fown) is
// added by the part that starts at slot 0.
template <int NT, bool VIR>
__device__ __forceinline__ void gather_bead(const GatherArgs &a, const Cut &cut, const int i, const float4 &pi,
                                            const int ti, float &Fx, float &Fy, float &Fz,
                                            float W[9], int &nR_in, int &nA_in, int p0 = 0, int step = 1) {
    const int n = a.n;
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
    if (p0 == 0) {
        float4 fo = a.fown[i];
        Fx = fo.x;
        Fy = fo.y;
        Fz = fo.z;
    } else {
        Fx = Fy = Fz = 0.0f;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) W[c] = 0.0f;
    // the neighbour's coefficients and the angular partial are loaded where
    // they are used: loading them ahead as well costs more registers (and
    // occupancy) than it hides
    RowStream rs;
    rs.start(a.nbr, a.pos4, n, i, cR, p0, step);
    for (int p = p0; p < cR; p += step) {
        const PairGeom g = rs.next_geom(p, pi, a.box);
        const int tj = (NT == 1) ? 0 : g.tj;
        const int tp = ti * NT + tj;
        if (g.d2 < cut.rcR2[tp]) {
            ++nR_in;
            nA_in += (p < cA && g.d2 < cut.rcA2[tp]) ? 1 : 0;
            const float ir = __builtin_amdgcn_rsqf(g.d2);
            const float r = g.d2 * ir;
            const float inv = cut.inv_rcR[tp];
            const float t = r * inv;
            const float sp = sin_pi(t), cp = cos_pi(t);
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
            const float4 v0 = src[0], v1 = src[1], v2 = src[2];
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
        // dU_j/dr_ji, angular part: delivered by j for every pair inside r_c^A
        if (p < cA && g.d2 < cut.rcA2[tp]) {
            const float4 fj = a.angbuf[(size_t)p * n + i];
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

}  // namespace nep
