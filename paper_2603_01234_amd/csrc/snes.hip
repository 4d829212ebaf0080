// The training loop around the batched fitness evaluation (Sec. II.A): the
// paper optimises the NEP parameters with SNES, the separable natural
// evolution strategy of Schaul et al. (GECCO 2011), on a loss of energy,
// force and virial RMSEs with L1 and L2 regularisation.  Every step of a
// generation runs on the device:
//   k_snes_sample    z_k = mu + sigma s_k (s_k: standard normals, an input)
//   k_derive_tables  each candidate model's coefficient and network tables
//                    from its parameter vector (the arithmetic of
//                    nep_model_create, so a model loaded here equals one
//                    created on the host from the same vector, bit for bit)
//   (the persistent fitness kernel then gives the RMSEs of every candidate)
//   k_snes_loss      L_k = lambda_e RMSE_E + lambda_f RMSE_F + lambda_v RMSE_W
//                          + lambda_1 mean|z_k| + lambda_2 sqrt(mean z_k^2)
//   k_snes_update    ranks (lower loss first, ties by index, non-finite
//                    last), utilities u_r = max(0, ln(lambda/2 + 1) - ln r) /
//                    sum - 1/lambda, natural gradients g_mu = sum_r u_r s_(r),
//                    g_sigma = sum_r u_r (s_(r)^2 - 1), and the updates
//                    mu += eta_mu sigma g_mu, sigma *= exp(eta_sigma/2 g_sigma).
#include "nep_internal.h"

namespace nep {

__global__ void k_snes_sample(int pop, size_t dim, const float *__restrict__ mu, const float *__restrict__ sigma,
                              const float *__restrict__ s, float *__restrict__ z) {
    const size_t total = (size_t)pop * dim;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const size_t p = t % dim;
        z[t] = mu[p] + sigma[p] * s[t];
    }
}

// one workgroup per model; entry e of the pair tables or of the network table
__global__ void k_derive_tables(DeriveArgs a) {
    const int m = blockIdx.x;
    const float *P = a.params + (size_t)m * a.n_params;
    const int T = a.T, H = a.H, HP = a.HP;
    const size_t D = ND;
    const float *cR = P + (size_t)T * H * D + 2 * (size_t)T * H + 1;
    const float *cA = cR + (size_t)T * T * NR * KB;
    float *tab = a.tab[m];
    float *ann = a.ann[m];
    float *flat = a.flat[m];
    for (size_t k = threadIdx.x; k < a.n_params; k += blockDim.x) flat[k] = P[k];
    const int ntab = T * T * TAB_PER_PAIR;
    for (int e = threadIdx.x; e < ntab; e += blockDim.x) {
        const int tp = e / TAB_PER_PAIR, o = e % TAB_PER_PAIR;
        const float *r = cR + (size_t)tp * NR * KB;
        const float *ang = cA + (size_t)tp * NA * KB;
        float v;
        if (o < NR * KB) {
            // radial: k = 0 carries c_n0 + sum_k c_nk  (f_k = hfc (T_k + 1))
            const int q = o / KB, k = o % KB;
            if (k == 0) {
                double s = 0.0;
                for (int kk = 0; kk < KB; ++kk) s += (double)r[q * KB + kk];
                v = (float)((double)r[q * KB] + s);
            } else {
                v = r[q * KB + k];
            }
        } else {
            const int oo = o - NR * KB, q = oo / KB, k = oo % KB;
            if (k == 0) {
                double s = 0.0;
                for (int kk = 0; kk < KB; ++kk) s += (double)ang[q * KB + kk];
                v = (float)((double)ang[q * KB] + s);
            } else {
                v = ang[q * KB + k];
            }
        }
        tab[e] = v;
    }
    // network per centre type: w0 transposed to [nu][mu], b0, w1, zero-padded to HP; then b1
    const int nann = T * (ND + 2) * HP;
    const float *w0 = P;
    const float *b0 = P + (size_t)T * H * D;
    const float *w1 = b0 + (size_t)T * H;
    for (int e = threadIdx.x; e <= nann; e += blockDim.x) {
        float v = 0.0f;
        if (e == nann) {
            v = w1[(size_t)T * H];
        } else {
            const int t = e / ((ND + 2) * HP), rem = e % ((ND + 2) * HP), row = rem / HP, mu = rem % HP;
            if (mu < H) {
                if (row < ND) v = w0[((size_t)t * H + mu) * D + row];
                else if (row == ND) v = b0[(size_t)t * H + mu];
                else v = w1[(size_t)t * H + mu];
            }
        }
        ann[e] = v;
    }
}

// one workgroup per candidate: loss from its RMSEs and its parameters
__global__ __launch_bounds__(BLOCK) void k_snes_loss(int pop, size_t dim, const float *__restrict__ z,
                                                     const double *__restrict__ rmse, nep_snes_params h,
                                                     double *__restrict__ loss) {
    __shared__ double red[2][BLOCK];
    const int k = blockIdx.x;
    const float *zk = z + (size_t)k * dim;
    double a1 = 0.0, a2 = 0.0;
    for (size_t p = threadIdx.x; p < dim; p += BLOCK) {
        const double v = (double)zk[p];
        a1 += fabs(v);
        a2 += v * v;
    }
    red[0][threadIdx.x] = a1;
    red[1][threadIdx.x] = a2;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double *r = rmse + 3 * (size_t)k;
        loss[k] = h.lambda_e * r[0] + h.lambda_f * r[1] + h.lambda_v * r[2] + h.lambda_1 * red[0][0] / (double)dim +
                  h.lambda_2 * sqrt(red[1][0] / (double)dim);
    }
}

constexpr int SNES_MAX_POP = 1024;

// grid over the parameters; every workgroup ranks the candidates (a few
// thousand comparisons) and builds the utilities itself
__global__ __launch_bounds__(BLOCK) void k_snes_update(int pop, size_t dim, const float *__restrict__ s,
                                                       const double *__restrict__ loss, nep_snes_params h,
                                                       float *__restrict__ mu, float *__restrict__ sigma,
                                                       int32_t *__restrict__ order_out) {
    __shared__ double L[SNES_MAX_POP];
    __shared__ double u[SNES_MAX_POP];
    __shared__ int order[SNES_MAX_POP];
    __shared__ double usum;
    for (int k = threadIdx.x; k < pop; k += BLOCK) {
        const double v = loss[k];
        L[k] = isfinite(v) ? v : INFINITY;
    }
    __syncthreads();
    const double lg = log(pop / 2.0 + 1.0);
    for (int k = threadIdx.x; k < pop; k += BLOCK) {
        int rank = 0;
        for (int j = 0; j < pop; ++j) rank += (L[j] < L[k] || (L[j] == L[k] && j < k)) ? 1 : 0;
        order[rank] = k;
        u[k] = fmax(0.0, lg - log((double)(k + 1)));   // raw utility of rank k (0-based)
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int r = 0; r < pop; ++r) t += u[r];
        usum = t;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < pop; r += BLOCK) u[r] = u[r] / usum - 1.0 / pop;
    __syncthreads();
    if (blockIdx.x == 0 && order_out)
        for (int r = threadIdx.x; r < pop; r += BLOCK) order_out[r] = order[r];
    const size_t p = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= dim) return;
    double gm = 0.0, gs = 0.0;
    for (int r = 0; r < pop; ++r) {
        const double v = (double)s[(size_t)order[r] * dim + p];
        gm += u[r] * v;
        gs += u[r] * (v * v - 1.0);
    }
    const double sg = (double)sigma[p];
    mu[p] = (float)((double)mu[p] + h.eta_mu * sg * gm);
    sigma[p] = (float)(sg * exp(0.5 * h.eta_sigma * gs));
}

hipError_t launch_snes_sample(int pop, size_t dim, const float *mu, const float *sigma, const float *s, float *z,
                              hipStream_t st) {
    const size_t total = (size_t)pop * dim;
    if (total == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>((total + BLOCK - 1) / BLOCK, 4096);
    hipLaunchKernelGGL(k_snes_sample, dim3(grid), dim3(BLOCK), 0, st, pop, dim, mu, sigma, s, z);
    return hipGetLastError();
}

hipError_t launch_derive_tables(const DeriveArgs &a, int n_models, hipStream_t st) {
    if (n_models == 0) return hipSuccess;
    hipLaunchKernelGGL(k_derive_tables, dim3(n_models), dim3(BLOCK), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_snes_update(int pop, size_t dim, const float *s, const float *z, const double *rmse,
                              const nep_snes_params &h, float *mu, float *sigma, double *loss, int32_t *order,
                              hipStream_t st) {
    if (pop == 0) return hipSuccess;
    hipLaunchKernelGGL(k_snes_loss, dim3(pop), dim3(BLOCK), 0, st, pop, dim, z, rmse, h, loss);
    const int grid = (int)((dim + BLOCK - 1) / BLOCK);
    if (grid > 0)
        hipLaunchKernelGGL(k_snes_update, dim3(grid), dim3(BLOCK), 0, st, pop, dim, s, loss, h, mu, sigma, order);
    return hipGetLastError();
}

}  // namespace nep
