// Learned per-column correction: coarsening, column features, a three-layer
// perceptron trained and evaluated with BF16 matrix-core (MFMA) products and
// FP32 accumulation, Adam in FP32, and the application of the predicted
// tendencies to a coarse state.
//
// Matrix products use gfx950's v_mfma_f32_16x16x32_bf16: one instruction
// adds a 16 x 32 by 32 x 16 BF16 product to a 16 x 16 FP32 tile.  Operand strides are explicit so the
// transposed products of the backward pass (X^T dZ, dZ W^T) read the stored
// row-major matrices in place.  The network is small (395 -> 256 -> 256 ->
// 237), so these are plain register-tiled products, not a library GEMM.
#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "fv3_internal.hpp"

namespace fv3 {

#define DEVI __device__ __forceinline__

typedef uint16_t bf16_t;
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// round to nearest even, the bit-exact rounding the oracle applies
DEVI bf16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (bf16_t)((u >> 16) | 0x40);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (bf16_t)(u >> 16);
}
DEVI float from_bf16(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// --------------------------------------------------------------- GEMM
// C(m, n) = sum_k A(m, k) B(k, n) [+ bias(n)], with A(m, k) = A[m*sam + k*sak]
// and B(k, n) = B[k*sbk + n*sbn] (BF16), C row-major FP32 (ldc).  Optional
// epilogue: tanh, and a BF16 copy of the result (ldcb).
enum { GE_NONE = 0, GE_TANH = 1 };

// Block tile 64 x 64 (four wavefronts, 32 x 32 each = 2 x 2 MFMA tiles), K
// staged through LDS 32 at a time.  Operands are loaded with the thread
// index running along whichever of their two dimensions is contiguous, and
// stored in LDS k-contiguous (A as [m][k], B as [n][k]) so that each lane
// reads its eight k-consecutive values of an MFMA operand (lane group g of
// 16 lanes holds k = 8g .. 8g + 7 of its row or column) as one 16-byte word.
// Accumulation runs over K in ascending chunks of 32, one MFMA per chunk
// and output tile.
constexpr int GBM = 64, GBN = 64, GBK = 32, GKP = GBK + 8;

__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const bf16_t *A, long sam, long sak,
                                                   const bf16_t *Bm, long sbk, long sbn, const float *bias,
                                                   int epi, float *C, long ldc, bf16_t *Cb, long ldcb)
{
    __shared__ __align__(16) bf16_t sA[GBM * GKP];
    __shared__ __align__(16) bf16_t sB[GBN * GKP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int r = lane & 15, g = lane >> 4;
    v4f acc[2][2];
    for (int x = 0; x < 2; x++)
        for (int y = 0; y < 2; y++) acc[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
    const bool a_kc = sak == 1, b_nc = sbn == 1;
    for (int k0 = 0; k0 < K; k0 += GBK) {
        // A tile: 64 x 32, eight values per thread
        if (a_kc) {
            int m = tid >> 2, kq = (tid & 3) * 8;
            int gm = m0 + m;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int gk = k0 + kq + q;
                sA[m * GKP + kq + q] = (gm < M && gk < K) ? A[(long)gm * sam + gk] : (bf16_t)0;
            }
        } else {
            int kk = tid >> 3, mq = (tid & 7) * 8;
            int gk = k0 + kk;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int gm = m0 + mq + q;
                sA[(mq + q) * GKP + kk] = (gm < M && gk < K) ? A[(long)gm * sam + (long)gk * sak] : (bf16_t)0;
            }
        }
        // B tile: 32 x 64, stored [n][k]
        if (b_nc) {
            int kk = tid >> 3, nq = (tid & 7) * 8;
            int gk = k0 + kk;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int gn = n0 + nq + q;
                sB[(nq + q) * GKP + kk] = (gn < N && gk < K) ? Bm[(long)gk * sbk + gn] : (bf16_t)0;
            }
        } else {
            int nn = tid >> 2, kq = (tid & 3) * 8;
            int gn = n0 + nn;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int gk = k0 + kq + q;
                sB[nn * GKP + kq + q] = (gn < N && gk < K) ? Bm[(long)gk * sbk + (long)gn * sbn] : (bf16_t)0;
            }
        }
        __syncthreads();
        static_assert(GBK == 32, "one 16x16x32 MFMA per K chunk");
        {
            v8bf a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; x++) {
                const v8s va = *(const v8s *)(sA + (wm + 16 * x + r) * GKP + 8 * g);
                const v8s vb = *(const v8s *)(sB + (wn + 16 * x + r) * GKP + 8 * g);
                a[x] = __builtin_bit_cast(v8bf, va);
                b[x] = __builtin_bit_cast(v8bf, vb);
            }
#pragma unroll
            for (int x = 0; x < 2; x++)
#pragma unroll
                for (int y = 0; y < 2; y++) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane holds rows 4g..4g+3 of column r of each 16 x 16 tile
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int m = m0 + wm + 16 * x + 4 * g + q, n = n0 + wn + 16 * y + r;
                if (m >= M || n >= N) continue;
                float v = acc[x][y][q] + (bias ? bias[n] : 0.f);
                if (epi == GE_TANH) v = tanhf(v);
                if (C) C[(long)m * ldc + n] = v;
                if (Cb) Cb[(long)m * ldcb + n] = to_bf16(v);
            }
}

static void gemm(int M, int N, int K, const bf16_t *A, long sam, long sak, const bf16_t *B, long sbk, long sbn,
                 const float *bias, int epi, float *C, long ldc, bf16_t *Cb, long ldcb, hipStream_t st)
{
    dim3 grd((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM));
    hipLaunchKernelGGL(k_gemm_bf16, grd, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, bias, epi, C, ldc,
                       Cb, ldcb);
}

// ------------------------------------------------------------ elementwise
__global__ void k_to_bf16(const float *x, long ldx, int rows, int cols, int cols_pad, bf16_t *y, long ldy)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols_pad) return;
    int r = (int)(e / cols_pad), c = (int)(e % cols_pad);
    y[(long)r * ldy + c] = c < cols ? to_bf16(x[(long)r * ldx + c]) : (bf16_t)0;
}

// dY = 2 (Y - T) / count on the true output columns, its BF16 copy, and the
// per-row squared error
__global__ void k_loss_grad(const float *Y, const float *T, int rows, int out, int out_pad, float scale,
                            float *dY, bf16_t *dYb, float *sq)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * out_pad) return;
    int r = (int)(e / out_pad), c = (int)(e % out_pad);
    float d = 0.f;
    if (c < out) {
        float res = Y[(long)r * out_pad + c] - T[(long)r * out + c];
        d = scale * res;
        atomicAdd(sq + (r & 1023), res * res);
    }
    dY[e] = d;
    dYb[e] = to_bf16(d);
}

// dZ = dH * (1 - H^2) (tanh derivative) and its BF16 copy
__global__ void k_tanh_back(const float *dH, const float *Hh, long count, float *dZ, bf16_t *dZb)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float h = Hh[e];
    float d = dH[e] * (1.f - h * h);
    dZ[e] = d;
    dZb[e] = to_bf16(d);
}

// column sums (bias gradients) in two deterministic passes: partial sums of
// 256-row chunks (threads along columns, coalesced), then the chunks in order
__global__ void k_colsum_partial(const float *x, int rows, int cols, long ld, float *part)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    int r0 = blockIdx.y * 256, r1 = min(rows, r0 + 256);
    float s = 0.f;
    for (int r = r0; r < r1; r++) s += x[(long)r * ld + c];
    part[(long)blockIdx.y * cols + c] = s;
}

__global__ void k_colsum_final(const float *part, int chunks, int cols, float *out)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int q = 0; q < chunks; q++) s += part[(long)q * cols + c];
    out[c] = s;
}

// Adam on FP32 master parameters; refresh the BF16 copy
__global__ void k_adam(float *p, const float *g, float *m, float *v, long count, float lr, float b1, float b2,
                       float eps, float c1, float c2, bf16_t *pb)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float gg = g[e];
    float mm = b1 * m[e] + (1.f - b1) * gg;
    float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    float mh = mm / c1, vh = vv / c2;
    float pn = p[e] - lr * mh / (sqrtf(vh) + eps);
    p[e] = pn;
    if (pb) pb[e] = to_bf16(pn);
}

__global__ void k_f32_to_bf16(const float *x, long count, bf16_t *y)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) y[e] = to_bf16(x[e]);
}

static unsigned nb(long count) { return (unsigned)((count + 255) / 256); }

}  // namespace fv3

// ====================================================================
// network object
// ====================================================================
struct fv3_mlp {
    int in, h1, h2, out;        // true sizes
    int inp, outp;              // padded to multiples of 16
    int maxrows;
    long step;
    // FP32 master parameters (padded layouts), Adam moments, BF16 copies
    float *W[3], *b[3], *mW[3], *vW[3], *mb[3], *vb[3], *gW[3], *gb[3];
    fv3::bf16_t *Wb[3];
    // activations and gradients for up to maxrows rows
    fv3::bf16_t *Xb, *H1b, *H2b, *dYb, *dZ2b, *dZ1b;
    float *H1, *H2, *Y, *dY, *dH2, *dZ2, *dH1, *dZ1, *sq, *part;
    int device;
};

namespace fv3 {
namespace {

long wrows(const fv3_mlp *n, int l) { return l == 0 ? n->inp : (l == 1 ? n->h1 : n->h2); }
long wcols(const fv3_mlp *n, int l) { return l == 0 ? n->h1 : (l == 1 ? n->h2 : n->outp); }

template <class T>
bool dalloc(T **p, long count)
{
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) return false;
    return hipMemset(*p, 0, count * sizeof(T)) == hipSuccess;
}

void colsum(fv3_mlp *n, const float *x, int rows, int cols, float *out, hipStream_t st)
{
    int chunks = (rows + 255) / 256;
    hipLaunchKernelGGL(k_colsum_partial, dim3((unsigned)((cols + 63) / 64), (unsigned)chunks), dim3(64), 0, st, x,
                       rows, cols, (long)cols, n->part);
    hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)((cols + 63) / 64)), dim3(64), 0, st, (const float *)n->part,
                       chunks, cols, out);
}

// forward pass on `rows` rows of X (FP32, in columns, row stride in)
void forward(fv3_mlp *n, const float *X, int rows, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(nb((long)rows * n->inp)), dim3(256), 0, st, X, (long)n->in, rows, n->in,
                       n->inp, n->Xb, (long)n->inp);
    gemm(rows, n->h1, n->inp, n->Xb, n->inp, 1, n->Wb[0], n->h1, 1, n->b[0], GE_TANH, n->H1, n->h1, n->H1b, n->h1, st);
    gemm(rows, n->h2, n->h1, n->H1b, n->h1, 1, n->Wb[1], n->h2, 1, n->b[1], GE_TANH, n->H2, n->h2, n->H2b, n->h2, st);
    gemm(rows, n->outp, n->h2, n->H2b, n->h2, 1, n->Wb[2], n->outp, 1, n->b[2], GE_NONE, n->Y, n->outp, nullptr, 0,
         st);
}

// gradients of the mean squared error over rows x out into gW, gb
void backward(fv3_mlp *n, const float *T, int rows, hipStream_t st)
{
    float scale = 2.0f / (float)((long)rows * n->out);
    (void)hipMemsetAsync(n->sq, 0, 1024 * sizeof(float), st);
    hipLaunchKernelGGL(k_loss_grad, dim3(nb((long)rows * n->outp)), dim3(256), 0, st, n->Y, T, rows, n->out,
                       n->outp, scale, n->dY, n->dYb, n->sq);
    // layer 3
    gemm(n->h2, n->outp, rows, n->H2b, 1, n->h2, n->dYb, n->outp, 1, nullptr, GE_NONE, n->gW[2], n->outp, nullptr, 0,
         st);
    colsum(n, n->dY, rows, n->outp, n->gb[2], st);
    gemm(rows, n->h2, n->outp, n->dYb, n->outp, 1, n->Wb[2], 1, n->outp, nullptr, GE_NONE, n->dH2, n->h2, nullptr,
         0, st);
    hipLaunchKernelGGL(k_tanh_back, dim3(nb((long)rows * n->h2)), dim3(256), 0, st, n->dH2, n->H2,
                       (long)rows * n->h2, n->dZ2, n->dZ2b);
    // layer 2
    gemm(n->h1, n->h2, rows, n->H1b, 1, n->h1, n->dZ2b, n->h2, 1, nullptr, GE_NONE, n->gW[1], n->h2, nullptr, 0, st);
    colsum(n, n->dZ2, rows, n->h2, n->gb[1], st);
    gemm(rows, n->h1, n->h2, n->dZ2b, n->h2, 1, n->Wb[1], 1, n->h2, nullptr, GE_NONE, n->dH1, n->h1, nullptr, 0, st);
    hipLaunchKernelGGL(k_tanh_back, dim3(nb((long)rows * n->h1)), dim3(256), 0, st, n->dH1, n->H1,
                       (long)rows * n->h1, n->dZ1, n->dZ1b);
    // layer 1
    gemm(n->inp, n->h1, rows, n->Xb, 1, n->inp, n->dZ1b, n->h1, 1, nullptr, GE_NONE, n->gW[0], n->h1, nullptr, 0, st);
    colsum(n, n->dZ1, rows, n->h1, n->gb[0], st);
}

}  // namespace
}  // namespace fv3

using namespace fv3;

namespace {
fv3_status mfail(fv3_status s, const char *m) { return set_error(s, m); }

bool on_device(const fv3_mlp *n)
{
    int cur = -1;
    return hipGetDevice(&cur) == hipSuccess && cur == n->device;
}
}  // namespace

extern "C" {

fv3_status fv3_mlp_create(int in, int h1, int h2, int out, int maxrows, const float *params, fv3_mlp **outp)
{
    if (!outp || !params || in < 1 || h1 < 16 || h2 < 16 || out < 1 || maxrows < 1 || (h1 % 16) || (h2 % 16))
        return mfail(FV3_EINVAL, "bad network sizes (hidden widths must be multiples of 16)");
    fv3_mlp *n = new fv3_mlp();
    n->in = in; n->h1 = h1; n->h2 = h2; n->out = out;
    n->inp = (in + 15) / 16 * 16;
    n->outp = (out + 15) / 16 * 16;
    n->maxrows = (maxrows + 15) / 16 * 16;
    n->step = 0;
    if (hipGetDevice(&n->device) != hipSuccess) {
        delete n;
        return mfail(FV3_EDEVICE, "no current HIP device");
    }
    bool ok = true;
    for (int l = 0; l < 3; l++) {
        long wc = wrows(n, l) * wcols(n, l), bc = wcols(n, l);
        ok = ok && dalloc(&n->W[l], wc) && dalloc(&n->mW[l], wc) && dalloc(&n->vW[l], wc) && dalloc(&n->gW[l], wc) &&
             dalloc(&n->b[l], bc) && dalloc(&n->mb[l], bc) && dalloc(&n->vb[l], bc) && dalloc(&n->gb[l], bc) &&
             dalloc(&n->Wb[l], wc);
    }
    long R = n->maxrows;
    ok = ok && dalloc(&n->Xb, R * n->inp) && dalloc(&n->H1b, R * h1) && dalloc(&n->H2b, R * h2) &&
         dalloc(&n->dYb, R * n->outp) && dalloc(&n->dZ2b, R * h2) && dalloc(&n->dZ1b, R * h1) &&
         dalloc(&n->H1, R * h1) && dalloc(&n->H2, R * h2) && dalloc(&n->Y, R * n->outp) &&
         dalloc(&n->dY, R * n->outp) && dalloc(&n->dH2, R * h2) && dalloc(&n->dZ2, R * h2) &&
         dalloc(&n->dH1, R * h1) && dalloc(&n->dZ1, R * h1) && dalloc(&n->sq, 1024) &&
         dalloc(&n->part, (R / 256 + 1) * (long)std::max(std::max(h1, h2), n->outp));
    if (!ok) {
        fv3_mlp_free(n);
        return mfail(FV3_ENOMEM, "device allocation failed");
    }
    *outp = n;
    fv3_status s = fv3_mlp_set_params(n, params);
    if (s != FV3_OK) {
        fv3_mlp_free(n);
        *outp = nullptr;
    }
    return s;
}

fv3_status fv3_mlp_free(fv3_mlp *n)
{
    if (!n) return FV3_OK;
    (void)hipDeviceSynchronize();
    for (int l = 0; l < 3; l++) {
        void *ps[] = {n->W[l], n->b[l], n->mW[l], n->vW[l], n->mb[l], n->vb[l], n->gW[l], n->gb[l], n->Wb[l]};
        for (void *p : ps)
            if (p) (void)hipFree(p);
    }
    void *ps[] = {n->Xb, n->H1b, n->H2b, n->dYb, n->dZ2b, n->dZ1b, n->H1, n->H2, n->Y, n->dY,
                  n->dH2, n->dZ2, n->dH1, n->dZ1, n->sq, n->part};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete n;
    return FV3_OK;
}

// packed parameter order: W1 (in x h1), b1, W2 (h1 x h2), b2, W3 (h2 x out), b3, row-major, unpadded
static long packed_count(const fv3_mlp *n)
{
    return (long)n->in * n->h1 + n->h1 + (long)n->h1 * n->h2 + n->h2 + (long)n->h2 * n->out + n->out;
}

fv3_status fv3_mlp_set_params(fv3_mlp *n, const float *params)
{
    if (!n || !params) return mfail(FV3_EINVAL, "NULL argument");
    const float *p = params;
    int tin[3] = {n->in, n->h1, n->h2}, tout[3] = {n->h1, n->h2, n->out};
    for (int l = 0; l < 3; l++) {
        long R = wrows(n, l), Cc = wcols(n, l);
        std::vector<float> w(R * Cc, 0.f), b(Cc, 0.f);
        for (int r = 0; r < tin[l]; r++)
            for (int c = 0; c < tout[l]; c++) w[r * Cc + c] = *p++;
        for (int c = 0; c < tout[l]; c++) b[c] = *p++;
        if (hipMemcpy(n->W[l], w.data(), w.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(n->b[l], b.data(), b.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return mfail(FV3_EDEVICE, "parameter upload failed");
        hipLaunchKernelGGL(k_f32_to_bf16, dim3(nb(R * Cc)), dim3(256), 0, 0, (const float *)n->W[l], R * Cc, n->Wb[l]);
        (void)hipMemset(n->mW[l], 0, R * Cc * 4);
        (void)hipMemset(n->vW[l], 0, R * Cc * 4);
        (void)hipMemset(n->mb[l], 0, Cc * 4);
        (void)hipMemset(n->vb[l], 0, Cc * 4);
    }
    n->step = 0;
    return hipDeviceSynchronize() == hipSuccess ? FV3_OK : mfail(FV3_EDEVICE, "sync failed");
}

fv3_status fv3_mlp_get_params(const fv3_mlp *n, float *params)
{
    if (!n || !params) return mfail(FV3_EINVAL, "NULL argument");
    if (hipDeviceSynchronize() != hipSuccess) return mfail(FV3_EDEVICE, "sync failed");
    float *p = params;
    int tin[3] = {n->in, n->h1, n->h2}, tout[3] = {n->h1, n->h2, n->out};
    for (int l = 0; l < 3; l++) {
        long R = wrows(n, l), Cc = wcols(n, l);
        std::vector<float> w(R * Cc), b(Cc);
        if (hipMemcpy(w.data(), n->W[l], w.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(b.data(), n->b[l], b.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return mfail(FV3_EDEVICE, "parameter download failed");
        for (int r = 0; r < tin[l]; r++)
            for (int c = 0; c < tout[l]; c++) *p++ = w[r * Cc + c];
        for (int c = 0; c < tout[l]; c++) *p++ = b[c];
    }
    return FV3_OK;
}

long fv3_mlp_param_count(const fv3_mlp *n) { return n ? packed_count(n) : 0; }

fv3_status fv3_mlp_forward(fv3_mlp *n, const float *X, int rows, float *Y, void *stream)
{
    if (!n || !X || !Y || rows < 1 || rows > n->maxrows) return mfail(FV3_EINVAL, "bad arguments");
    if (!on_device(n)) return mfail(FV3_EDEVICE, "current HIP device differs from the network's device");
    hipStream_t st = (hipStream_t)stream;
    forward(n, X, rows, st);
    // copy the true output columns out
    if (hipMemcpy2DAsync(Y, (size_t)n->out * 4, n->Y, (size_t)n->outp * 4, (size_t)n->out * 4, rows,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
        return mfail(FV3_EDEVICE, "output copy failed");
    return FV3_OK;
}

fv3_status fv3_mlp_gradients(fv3_mlp *n, const float *X, const float *T, int rows, float *grads, void *stream)
{
    if (!n || !X || !T || !grads || rows < 1 || rows > n->maxrows) return mfail(FV3_EINVAL, "bad arguments");
    if (!on_device(n)) return mfail(FV3_EDEVICE, "current HIP device differs from the network's device");
    hipStream_t st = (hipStream_t)stream;
    forward(n, X, rows, st);
    backward(n, T, rows, st);
    if (hipStreamSynchronize(st) != hipSuccess) return mfail(FV3_EDEVICE, "sync failed");
    float *p = grads;
    int tin[3] = {n->in, n->h1, n->h2}, tout[3] = {n->h1, n->h2, n->out};
    for (int l = 0; l < 3; l++) {
        long R = wrows(n, l), Cc = wcols(n, l);
        std::vector<float> w(R * Cc), b(Cc);
        if (hipMemcpy(w.data(), n->gW[l], w.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(b.data(), n->gb[l], b.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return mfail(FV3_EDEVICE, "gradient download failed");
        for (int r = 0; r < tin[l]; r++)
            for (int c = 0; c < tout[l]; c++) *p++ = w[r * Cc + c];
        for (int c = 0; c < tout[l]; c++) *p++ = b[c];
    }
    return FV3_OK;
}

fv3_status fv3_mlp_train_step(fv3_mlp *n, const float *X, const float *T, int rows, float lr, double *loss,
                              void *stream)
{
    if (!n || !X || !T || rows < 1 || rows > n->maxrows) return mfail(FV3_EINVAL, "bad arguments");
    if (!on_device(n)) return mfail(FV3_EDEVICE, "current HIP device differs from the network's device");
    hipStream_t st = (hipStream_t)stream;
    forward(n, X, rows, st);
    backward(n, T, rows, st);
    n->step++;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float c1 = 1.f - powf(b1, (float)n->step), c2 = 1.f - powf(b2, (float)n->step);
    for (int l = 0; l < 3; l++) {
        long wc = wrows(n, l) * wcols(n, l), bc = wcols(n, l);
        hipLaunchKernelGGL(k_adam, dim3(nb(wc)), dim3(256), 0, st, n->W[l], (const float *)n->gW[l], n->mW[l],
                           n->vW[l], wc, lr, b1, b2, eps, c1, c2, n->Wb[l]);
        hipLaunchKernelGGL(k_adam, dim3(nb(bc)), dim3(256), 0, st, n->b[l], (const float *)n->gb[l], n->mb[l],
                           n->vb[l], bc, lr, b1, b2, eps, c1, c2, (bf16_t *)nullptr);
    }
    if (loss) {
        std::vector<float> sq(1024);
        if (hipMemcpyAsync(sq.data(), n->sq, 1024 * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return mfail(FV3_EDEVICE, "loss read failed");
        double s = 0.0;
        for (float x : sq) s += x;
        *loss = s / ((double)rows * n->out);
    }
    return hipGetLastError() == hipSuccess ? FV3_OK : mfail(FV3_EDEVICE, "launch failed");
}

}  // extern "C"
