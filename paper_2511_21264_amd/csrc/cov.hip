// Covariance adaptation and full-covariance sampling (Alg. 1: sampling from
// N(nu_m, Sigma_m); Eqs. mean_update and cov_update with the weights of
// Eq. s_formula).  A sequence is the n = 14 H vector of its joint velocities
// in step-major order (index 14 k + d), so Sigma is n x n, row-major, FP64.
//
//   cov_syrk_kernel    Sigma' = (1 - eta) Sigma + eta sum_j w_j D_j D_j^T / sum w
//                      + eps I with D_j = u_j - nu_{m+1}: one workgroup per
//                      32 x 32 lower tile, the four waves split the samples,
//                      FP64 MFMA 16x16x4 with the deviation and the weight
//                      formed in the operand load; each symmetric pair is
//                      written by one lane (so the update may run in place)
//   chol_*_kernel      blocked right-looking Cholesky in FP64, 32-wide block
//                      columns, one launch per block column: every trailing
//                      lower tile (r, c) forms the panel blocks A_rb L_bb^-T
//                      and A_cb L_bb^-T itself and subtracts their product
//                      (FP64 MFMA); the tile (r, r) also stores its panel block
//                      as the factor, and the workgroup of the next diagonal
//                      tile factors and inverts it in registers once updated
//   sample_full_kernel U = clip(nu + Z L^T, +-u_max): FP32 MFMA 16x16x4 over
//                      16 x 64 tiles staged through LDS in 32-wide chunks,
//                      skipping the zero upper triangle of L
//
// MFMA 16x16x4 operand layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; result element v of lane l is D[4 (l / 16) + v][l % 16]
// for f32 and D[l / 16 + 4 v][l % 16] for f64 (measured on gfx950).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "team.h"

namespace mppi {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int CT = 32;  // covariance output tile edge
constexpr int CB = 32;  // Cholesky block edge

// t -> (row, col) of the t-th lower tile, enumerated row by row
__device__ __forceinline__ void tri_index(int t, int &row, int &col)
{
    int b = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
    while (b * (b + 1) / 2 > t) --b;
    while ((b + 1) * (b + 2) / 2 <= t) ++b;
    row = b;
    col = t - b * (b + 1) / 2;
}

// Workgroups are dealt to the eight XCDs (each with its own L2) in turn by
// their index b; this maps b to a logical tile so that every XCD takes one
// contiguous range of tiles (a bijection on 0 .. nb - 1): tiles that share
// input rows then share an L2.
__device__ __forceinline__ int xcd_order(int b, int nb)
{
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + (b >> 3);
}

__device__ __forceinline__ double wave_sum_f64(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

}  // namespace

// ------------------------------------------------------------ covariance update
constexpr int CG = 8;  // groups of four samples per wave and step

__global__ void __launch_bounds__(256) cov_syrk_kernel(CovArgs a)
{
    __shared__ double red[4][CT][CT + 1];
    __shared__ double wred[4];
    int bi, bl;
    tri_index(xcd_order(blockIdx.x, gridDim.x), bi, bl);  // consecutive rows of tiles share an XCD
    const int n = a.n, K = a.K;
    const int i0 = bi * CT, l0 = bl * CT;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int ia0 = i0 + r, ia1 = ia0 + 16, lb0 = l0 + r, lb1 = lb0 + 16;
    const double na0 = ia0 < n ? a.nu[ia0] : 0.0, na1 = ia1 < n ? a.nu[ia1] : 0.0;
    const double nl0 = lb0 < n ? a.nu[lb0] : 0.0, nl1 = lb1 < n ? a.nu[lb1] : 0.0;
    d4 c00 = {0.0, 0.0, 0.0, 0.0}, c01 = c00, c10 = c00, c11 = c00;
    double ws = 0.0;
    // wave wv takes the groups of four samples j0 = 4 wv, 4 wv + 16, ...,
    // CG groups per step; the loads of step s + 1 are issued before the
    // products of step s.  Sample values do not wait on their weight: a
    // weightless sample is dropped by a select afterwards (so a non-finite
    // entry in it still contributes nothing).
    float uc[CG][4], un[CG][4] = {};
    double wc[CG], wn[CG] = {};
    auto load = [&](int j0, float (&u4)[CG][4], double (&w2)[CG]) {
#pragma unroll
        for (int g = 0; g < CG; ++g) {
            const int j = j0 + 16 * g + q;
            const bool ok = j < K;
            const float *u = a.U + (long)(ok ? j : 0) * n;
            w2[g] = ok ? a.w[j] : 0.0;
            u4[g][0] = (ok && ia0 < n) ? u[ia0] : 0.f;
            u4[g][1] = (ok && ia1 < n) ? u[ia1] : 0.f;
            u4[g][2] = (ok && lb0 < n) ? u[lb0] : 0.f;
            u4[g][3] = (ok && lb1 < n) ? u[lb1] : 0.f;
        }
    };
    load(4 * wv, uc, wc);
    for (int j0 = 4 * wv; j0 < K; j0 += 16 * CG) {
        if (j0 + 16 * CG < K) load(j0 + 16 * CG, un, wn);
        bool any = false;
#pragma unroll
        for (int g = 0; g < CG; ++g) {
            if (r == 0) ws += wc[g];
            any = any || wc[g] != 0.0;
        }
        if (__ballot(any) != 0) {  // skipped when no group of the step carries weight
#pragma unroll
            for (int g = 0; g < CG; ++g) {
                const bool on = wc[g] != 0.0;
                const double x0 = on ? (double)uc[g][0] - na0 : 0.0, x1 = on ? (double)uc[g][1] - na1 : 0.0;
                const double y0 = on ? wc[g] * ((double)uc[g][2] - nl0) : 0.0;
                const double y1 = on ? wc[g] * ((double)uc[g][3] - nl1) : 0.0;
                c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, c00, 0, 0, 0);
                c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, c01, 0, 0, 0);
                c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, c10, 0, 0, 0);
                c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, c11, 0, 0, 0);
            }
        }
#pragma unroll
        for (int g = 0; g < CG; ++g) {
            wc[g] = wn[g];
#pragma unroll
            for (int e = 0; e < 4; ++e) uc[g][e] = un[g][e];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        red[wv][q + 4 * v][r] = c00[v];
        red[wv][q + 4 * v][16 + r] = c01[v];
        red[wv][16 + q + 4 * v][r] = c10[v];
        red[wv][16 + q + 4 * v][16 + r] = c11[v];
    }
    ws = wave_sum_f64(ws);
    if (lane == 0) wred[wv] = ws;
    __syncthreads();
    const double wsum = ((wred[0] + wred[1]) + wred[2]) + wred[3];
    for (int e = threadIdx.x; e < CT * CT; e += 256) {
        const int ti = e / CT, tl = e % CT;
        const int i = i0 + ti, l = l0 + tl;
        if (i >= n || l >= n || (bi == bl && ti < tl)) continue;
        const double g = ((red[0][ti][tl] + red[1][ti][tl]) + red[2][ti][tl]) + red[3][ti][tl];
        const double s_old = a.S_in[(long)i * n + l];
        // no weight at all (no finite cost): Sigma is kept, as the mean is
        double v = s_old;
        if (wsum > 0.0) {
            v = (1.0 - a.eta) * s_old + a.eta * (g / wsum);
            if (i == l) v += a.eps;
        }
        a.S_out[(long)i * n + l] = v;
        red[0][ti][tl] = v;  // read above by this thread only
    }
    __syncthreads();
    // the mirrored upper half, written along its rows
    for (int e = threadIdx.x; e < CT * CT; e += 256) {
        const int tl = e / CT, ti = e % CT;
        const int i = i0 + ti, l = l0 + tl;
        if (i >= n || l >= n || i == l || (bi == bl && ti < tl)) continue;
        a.S_out[(long)l * n + i] = red[0][ti][tl];
    }
}

void launch_cov_update(const CovArgs &a, hipStream_t s)
{
    const int nt = (a.n + CT - 1) / CT;
    hipLaunchKernelGGL(cov_syrk_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, a);
}

// ------------------------------------------------------------------ Cholesky
__global__ void __launch_bounds__(256) chol_init_kernel(CholArgs a)
{
    const long n = a.n, N = n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
        const long i = e / n, l = e - i * n;
        if (l <= i) {
            a.A[e] = a.S[e];
        } else {
            a.L[e] = 0.0;
            if (a.L32) a.L32[e] = 0.f;
        }
    }
    if (a.reset_flag && blockIdx.x == 0 && threadIdx.x == 0) *a.flag = a.n;
}

// element i (0..3) of a four-vector without dynamic indexing (sum of
// selects: no lookup table, no scratch)
__device__ __forceinline__ double pick4(const double v[4], int i)
{
    return (i == 0 ? v[0] : 0.0) + (i == 1 ? v[1] : 0.0) + (i == 2 ? v[2] : 0.0) + (i == 3 ? v[3] : 0.0);
}

// Factor the diagonal block held in s (lower triangle valid for rows and
// columns < nbk), invert it, and store the factor block of columns c0.. into
// L (and L32) and the inverse into Linv.  256 threads: thread t keeps the
// entries (t / 32 + 8 k, t % 32), k = 0..3, of the block and of its inverse
// in registers.  Columns go four at a time: their owners publish them (and
// the four matching rows of the inverse) to LDS, one barrier, then every
// thread factors the 4 x 4 diagonal block itself, forms its rows of the
// panel by forward substitution and applies the rank-4 update to its
// entries; rows of X = L^-1 follow by forward elimination of L X = I.  The
// published panels alternate between two buffers, so one barrier per four
// columns suffices.
__device__ void factor_block(const double (*s)[CB + 1], double (*cbuf)[4][CB], double (*xbuf)[4][CB], int nbk,
                             int c0b, const CholArgs &a, double *Linv)
{
    const int t = threadIdx.x, q = t & 31, r0 = t >> 5;
    const int n = a.n;
    double sv[4], xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = r0 + 8 * k;
        if (r >= nbk || q >= nbk)
            sv[k] = r == q ? 1.0 : 0.0;  // rows and columns past n: the identity
        else
            sv[k] = q <= r ? s[r][q] : 0.0;
        xv[k] = r == q ? 1.0 : 0.0;
    }
    int bad = -1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int c0 = 4 * i, par = i & 1, kb = i >> 1;  // rows c0..c0+3 are k = kb of threads r0 = c0 & 7 ..
        if (q >= c0 && q < c0 + 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) cbuf[par][q - c0][r0 + 8 * k] = sv[k];
        }
        {
            const int rr = r0 + 8 * kb;
            if (rr >= c0 && rr < c0 + 4) xbuf[par][rr - c0][q] = xv[kb];
        }
        __syncthreads();
        // the 4 x 4 diagonal block, factored (left-looking) by every thread
        double L4[4][4], id[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double p = cbuf[par][u][c0 + u];
#pragma unroll
            for (int w = 0; w < u; ++w) p -= L4[u][w] * L4[u][w];
            if (bad < 0 && !(p > 0.0 && p < INFINITY)) bad = c0 + u;
            id[u] = rsqrt(p);
            L4[u][u] = p * id[u];
#pragma unroll
            for (int v = u + 1; v < 4; ++v) {
                double x = cbuf[par][u][c0 + v];
#pragma unroll
                for (int w = 0; w < u; ++w) x -= L4[v][w] * L4[u][w];
                L4[v][u] = x * id[u];
            }
        }
        // panel row r: l[u] = (a_r[u] - sum_{w<u} l[w] L4[u][w]) / L4[u][u]
        auto panel = [&](int r, double l[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                double x = cbuf[par][u][r];
#pragma unroll
                for (int w = 0; w < u; ++w) x -= l[w] * L4[u][w];
                l[u] = x * id[u];
            }
        };
        double lq[4], xc[4];
        panel(q, lq);
        // rows c0..c0+3 of X at column q
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double x = xbuf[par][u][q];
#pragma unroll
            for (int w = 0; w < u; ++w) x -= L4[u][w] * xc[w];
            xc[u] = x * id[u];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = r0 + 8 * k;
            double lr[4];
            panel(r, lr);
            if (r >= c0 + 4) {
                const double upd = ((sv[k] - lr[0] * lq[0]) - lr[1] * lq[1]) - lr[2] * lq[2] - lr[3] * lq[3];
                if (q >= c0 + 4 && q <= r)
                    sv[k] = upd;
                else if (q >= c0 && q < c0 + 4)
                    sv[k] = pick4(lr, q - c0);
                xv[k] = (((xv[k] - lr[0] * xc[0]) - lr[1] * xc[1]) - lr[2] * xc[2]) - lr[3] * xc[3];
            } else if (r >= c0) {
                const int u = r - c0;
                if (q >= c0 && q <= r) {
                    // L4[u][q - c0]: row u of the lower factor (entries above the diagonal are not read)
                    const double lu[4] = {u == 0 ? L4[0][0] : (u == 1 ? L4[1][0] : (u == 2 ? L4[2][0] : L4[3][0])),
                                          u == 1 ? L4[1][1] : (u == 2 ? L4[2][1] : L4[3][1]),
                                          u == 2 ? L4[2][2] : L4[3][2], L4[3][3]};
                    sv[k] = pick4(lu, q - c0);
                }
                xv[k] = pick4(xc, u);
            }
        }
    }
    if (t == 0 && bad >= 0 && bad < nbk && *a.flag == n) *a.flag = c0b + bad;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = r0 + 8 * k;
        Linv[r * CB + q] = xv[k];
        if (r < nbk && q <= r) {
            const long e = (long)(c0b + r) * n + c0b + q;
            a.L[e] = sv[k];
            if (a.L32) a.L32[e] = (float)sv[k];
        }
    }
}

// the first diagonal block (the others are factored by the step before them)
__global__ void __launch_bounds__(256) chol_diag_kernel(CholArgs a)
{
    __shared__ double s[CB][CB + 1];
    __shared__ double cbuf[2][4][CB], xbuf[2][4][CB];
    const int n = a.n, nbk = min(CB, n);
    for (int e = threadIdx.x; e < CB * CB; e += 256) {
        const int r = e / CB, q = e % CB;
        if (r < nbk && q <= r) s[r][q] = a.A[(long)r * n + q];
    }
    __syncthreads();
    factor_block(s, cbuf, xbuf, nbk, 0, a, a.Linv);
}

// Step b of the right-looking factorization over the trailing lower tiles
// (rb, cb), b < cb <= rb: P = A_blk L_bb^-T for block rows rb and cb, then
// A_{rb,cb} -= P_rb P_cb^T (FP64 MFMA, wave w: output block (w / 2, w % 2)).
// The tile (rb, rb) stores P_rb as the factor; the tile (b + 1, b + 1),
// complete after this update, is factored and inverted right away.  The
// inverse of block b is read from Linv[b & 1] and that of b + 1 written to
// the other half, so no workgroup of this launch reads what another writes.
__global__ void __launch_bounds__(256) chol_step_kernel(CholArgs a, int b)
{
    __shared__ double li[CB][CB + 1];
    __shared__ double ar[CB][CB + 1];
    __shared__ double ac[CB][CB + 1];
    __shared__ double pr[CB][CB + 1];
    __shared__ double pc[CB][CB + 1];
    __shared__ double cbuf[2][4][CB], xbuf[2][4][CB];
    int rr, cc;
    tri_index(blockIdx.x, rr, cc);
    const int rb = b + 1 + rr, cb = b + 1 + cc;
    const int n = a.n, c0 = b * CB, R0 = rb * CB, C0 = cb * CB;
    const bool diag = rb == cb;
    const double *Li = a.Linv + (b & 1) * CB * CB;
    for (int e = threadIdx.x; e < CB * CB; e += 256) {
        const int x = e / CB, y = e % CB;
        li[x][y] = Li[e];
        // block column b is whole: b < the last block column
        ar[x][y] = R0 + x < n ? a.A[(long)(R0 + x) * n + c0 + y] : 0.0;
        if (!diag) ac[x][y] = C0 + x < n ? a.A[(long)(C0 + x) * n + c0 + y] : 0.0;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lq = lane >> 4;
    const int ba = 16 * (wv >> 1), bb = 16 * (wv & 1);
    d4 c1 = {0.0, 0.0, 0.0, 0.0}, c2 = c1;
#pragma unroll
    for (int kk = 0; kk < CB; kk += 4) {
        const double y = li[bb + lr][kk + lq];
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ba + lr][kk + lq], y, c1, 0, 0, 0);
        if (!diag) c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[ba + lr][kk + lq], y, c2, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        pr[ba + lq + 4 * v][bb + lr] = c1[v];
        if (!diag) pc[ba + lq + 4 * v][bb + lr] = c2[v];
    }
    __syncthreads();
    double(*pcc)[CB + 1] = diag ? pr : pc;
    d4 cu = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < CB; kk += 4)
        cu = __builtin_amdgcn_mfma_f64_16x16x4f64(pr[ba + lr][kk + lq], pcc[bb + lr][kk + lq], cu, 0, 0, 0);
    const bool next = diag && rb == b + 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int x = ba + lq + 4 * v, y = bb + lr;
        if (R0 + x < n && C0 + y < n && (!diag || y <= x)) {
            const long e = (long)(R0 + x) * n + C0 + y;
            const double nv = a.A[e] - cu[v];
            a.A[e] = nv;
            if (next) ar[x][y] = nv;  // ar is no longer read: the products above are done
        }
    }
    if (diag) {
        for (int e = threadIdx.x; e < CB * CB; e += 256) {
            const int x = e / CB, y = e % CB;
            if (R0 + x >= n) continue;
            const long eL = (long)(R0 + x) * n + c0 + y;
            a.L[eL] = pr[x][y];
            if (a.L32) a.L32[eL] = (float)pr[x][y];
        }
    }
    if (next) {
        __syncthreads();
        factor_block(ar, cbuf, xbuf, min(CB, n - R0), R0, a, a.Linv + ((b + 1) & 1) * CB * CB);
    }
}

void launch_cholesky(const CholArgs &a, hipStream_t s)
{
    const long N = (long)a.n * a.n;
    const int g = (int)std::min<long>((N + 255) / 256, 4096);
    hipLaunchKernelGGL(chol_init_kernel, dim3(g), dim3(256), 0, s, a);
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, a);
    const int nb = (a.n + CB - 1) / CB;
    for (int b = 0; b + 1 < nb; ++b) {
        const int T = nb - b - 1;
        hipLaunchKernelGGL(chol_step_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, s, a, b);
    }
}

// ------------------------------------------------------------------ sampling
__global__ void __launch_bounds__(256) normals_kernel(SampleFullArgs a)
{
    const long n = a.n, N = (long)a.K * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
        const long j = e / n;
        const int i = (int)(e - j * n);
        a.Z[e] = normal_joint(a.key0, a.key1, (uint32_t)j, (uint32_t)(i / NU), (uint32_t)a.m, i % NU);
    }
}

// output tile: 16 samples (j) x 64 sequence entries (i); wave w owns entries
// i0 + 16 w .. + 15 (one 16x16 MFMA block); the sum over p runs in chunks of
// 32 columns staged through LDS.  Small tiles keep several workgroups per
// CU, whose loads overlap.
constexpr int SJ = 16, SI = 64, SP = 32;

__global__ void __launch_bounds__(256) sample_full_kernel(SampleFullArgs a)
{
    __shared__ float zs[SJ][SP + 1];
    __shared__ float ls[SI][SP + 1];
    const int n = a.n, K = a.K;
    // all column tiles of a block of samples on one XCD (their normals share its L2)
    const int ni = (n + SI - 1) / SI, tile = xcd_order(blockIdx.x, gridDim.x);
    const int i0 = (tile % ni) * SI, j0 = (tile / ni) * SJ;
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63, r = lane & 15, q = lane >> 4;
    f4 c0 = {0.f, 0.f, 0.f, 0.f};
    const int pend = min(n, i0 + SI);  // L is lower: columns past the tile's last row are zero
    // chunk p0 holds Z[j0.., p0..] (16 x 32) and L[i0.., p0..] (64 x 32):
    // thread t takes column t % 32; the next chunk is loaded into registers
    // while the current one is multiplied
    const int pc = t & 31, rw = t >> 5;
    float zr[SJ / 8], lr[SI / 8];
    auto load = [&](int p0) {
        const int p = p0 + pc;
#pragma unroll
        for (int u = 0; u < SJ / 8; ++u) {
            const int row = rw + 8 * u;
            zr[u] = (j0 + row < K && p < n) ? a.Z[(long)(j0 + row) * n + p] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < SI / 8; ++u) {
            const int row = rw + 8 * u;
            lr[u] = (i0 + row < n && p < n) ? a.L32[(long)(i0 + row) * n + p] : 0.f;
        }
    };
    load(0);
    for (int p0 = 0; p0 < pend; p0 += SP) {
#pragma unroll
        for (int u = 0; u < SJ / 8; ++u) zs[rw + 8 * u][pc] = zr[u];
#pragma unroll
        for (int u = 0; u < SI / 8; ++u) ls[rw + 8 * u][pc] = lr[u];
        __syncthreads();
        if (p0 + SP < pend) load(p0 + SP);
#pragma unroll
        for (int kk = 0; kk < SP / 4; ++kk)
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(zs[r][4 * kk + q], ls[16 * wv + r][4 * kk + q], c0, 0, 0, 0);
        __syncthreads();
    }
    const int ib = i0 + 16 * wv + r;
    const float nui = ib < n ? a.nu[ib] : 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int ja = j0 + 4 * q + v;
        if (ja < K && ib < n) a.U[(long)ja * n + ib] = fminf(fmaxf(nui + c0[v], -a.u_max), a.u_max);
    }
}

void launch_sample_full(const SampleFullArgs &a, hipStream_t s)
{
    const long N = (long)a.K * a.n;
    const int g = (int)std::min<long>((N + 255) / 256, 8192);
    hipLaunchKernelGGL(normals_kernel, dim3(g), dim3(256), 0, s, a);
    hipLaunchKernelGGL(sample_full_kernel, dim3(((a.n + SI - 1) / SI) * ((a.K + SJ - 1) / SJ)), dim3(256), 0, s, a);
}

__global__ void __launch_bounds__(256) diag_sigma_kernel(const float *sigma, int sps, int n, double *S)
{
    const long N = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
        const long i = e / n, l = e - i * n;
        double v = 0.0;
        if (i == l) {
            const double sg = sigma[sps ? i : i % NU];
            v = sg * sg;
        }
        S[e] = v;
    }
}

void launch_diag_sigma(const float *sigma, int sps, int n, double *S, hipStream_t s)
{
    const long N = (long)n * n;
    const int g = (int)std::min<long>((N + 255) / 256, 4096);
    hipLaunchKernelGGL(diag_sigma_kernel, dim3(g), dim3(256), 0, s, sigma, sps, n, S);
}

__global__ void __launch_bounds__(256) to_f32_kernel(const double *src, float *dst, long N)
{
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x)
        dst[e] = (float)src[e];
}

void launch_to_f32(const double *src, float *dst, long N, hipStream_t s)
{
    const int g = (int)std::min<long>((N + 255) / 256, 4096);
    hipLaunchKernelGGL(to_f32_kernel, dim3(g), dim3(256), 0, s, src, dst, N);
}

__global__ void __launch_bounds__(256) lower_f32_kernel(float *L, int n)
{
    const long N = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N; e += (long)gridDim.x * blockDim.x) {
        const long i = e / n, l = e - i * n;
        if (l > i) L[e] = 0.f;
    }
}

void launch_lower_f32(float *L, int n, hipStream_t s)
{
    const long N = (long)n * n;
    const int g = (int)std::min<long>((N + 255) / 256, 4096);
    hipLaunchKernelGGL(lower_f32_kernel, dim3(g), dim3(256), 0, s, L, n);
}

}  // namespace mppi
