// Contrastive losses of matched (image, text) batches and their gradients,
// FP32: logits l_ij = scale <e_i, t_j> + bias, then
//   softmax head (CLIP, Radford et al. 2021, Sec. 2.3): the mean of the
//     image->text and text->image cross-entropies with the matching pair as
//     the target,
//   sigmoid head (SigLIP, Zhai et al. 2023, Eq. 1): -(1/n) sum_ij log
//     sigmoid(z_ij l_ij), z_ij = +1 on the diagonal and -1 elsewhere.
// dL/dl (G) is formed element-wise from the logits and the row / column
// log-sum-exps; the embedding gradients are the GEMMs scale * G T and
// scale * G^T E.
#include <mutex>

#include "kernels.hpp"

namespace vl {

// Per-row log-sum-exp of L [n, ld] (first n columns).  One workgroup per row.
__global__ __launch_bounds__(256) void k_row_lse(const float* __restrict__ L, int n, int ld,
                                                 float* __restrict__ lse) {
  __shared__ float red[4];
  const float* r = L + (size_t)blockIdx.x * ld;
  float mx = -INFINITY;
  for (int j = threadIdx.x; j < n; j += 256) mx = fmaxf(mx, r[j]);
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  float s = 0.f;
  for (int j = threadIdx.x; j < n; j += 256) s += expf(r[j] - mx);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) lse[blockIdx.x] = mx + logf((red[0] + red[1]) + (red[2] + red[3]));
}

// Per-column log-sum-exp: a workgroup owns 64 columns; its 4 waves walk
// interleaved rows (coalesced 256-byte row segments) with a running max and
// sum each, merged at the end.
__global__ __launch_bounds__(256) void k_col_lse(const float* __restrict__ L, int n, int ld,
                                                 float* __restrict__ lse) {
  __shared__ float smx[4][64], ssum[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  float mx = -INFINITY, s = 0.f;
  if (c < n)
    for (int i = g; i < n; i += 4) {
      const float v = L[(size_t)i * ld + c];
      if (v > mx) {
        s = s * expf(mx - v) + 1.f;
        mx = v;
      } else {
        s += expf(v - mx);
      }
    }
  smx[g][threadIdx.x & 63] = mx;
  ssum[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && c < n) {
    const int l = threadIdx.x;
    const float m = fmaxf(fmaxf(smx[0][l], smx[1][l]), fmaxf(smx[2][l], smx[3][l]));
    float t = 0.f;
    for (int k = 0; k < 4; ++k) t += ssum[k][l] * expf(smx[k][l] - m);
    lse[c] = m + logf(t);
  }
}

// Row i of G = dL/dl, in place over L (columns n..ld-1 set to zero: they are
// the K padding of the gradient GEMMs), plus the row's contributions (loss,
// sum_j G_ij (l_ij - bias), sum_j G_ij) in part[3i..3i+2].
__global__ __launch_bounds__(256) void k_contrastive_grad(float* __restrict__ L, int n, int ld,
                                                          int head, float bias,
                                                          const float* __restrict__ rlse,
                                                          const float* __restrict__ clse,
                                                          float* __restrict__ part) {
  __shared__ float red[3][4];
  const int i = blockIdx.x;
  float* r = L + (size_t)i * ld;
  const float inv_n = 1.f / (float)n;
  float sl = 0.f, sg = 0.f, s0 = 0.f;
  for (int j = threadIdx.x; j < n; j += 256) {
    const float l = r[j];
    float g;
    if (head == 0) {
      const float d = j == i ? 1.f : 0.f;
      g = 0.5f * inv_n * ((expf(l - rlse[i]) - d) + (expf(l - clse[j]) - d));
    } else {
      const float z = j == i ? 1.f : -1.f;
      const float u = -z * l;                 // loss term softplus(u)
      sl += u > 0.f ? u + log1pf(expf(-u)) : log1pf(expf(u));
      g = -z * inv_n / (1.f + expf(-u));      // -z sigmoid(u) / n
    }
    r[j] = g;
    sg += g * (l - bias);
    s0 += g;
  }
  for (int j = n + threadIdx.x; j < ld; j += 256) r[j] = 0.f;
  sl = wave_sum(sl); sg = wave_sum(sg); s0 = wave_sum(s0);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sl; red[1][threadIdx.x >> 6] = sg; red[2][threadIdx.x >> 6] = s0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[3 * i + 0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    part[3 * i + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    part[3 * i + 2] = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
  }
}

// Softmax-head loss terms need the diagonal logits, which the gradient
// kernel overwrites: take them first.  diag[i] = l_ii.
__global__ void k_diag(const float* __restrict__ L, int n, int ld, float* __restrict__ diag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) diag[i] = L[(size_t)i * ld + i];
}

// Fixed-order reduction of the row partials into loss, dL/dscale, dL/dbias.
__global__ __launch_bounds__(256) void k_contrastive_reduce(const float* __restrict__ part,
                                                            const float* __restrict__ rlse,
                                                            const float* __restrict__ clse,
                                                            const float* __restrict__ diag, int n,
                                                            int head, float scale,
                                                            float* __restrict__ loss,
                                                            float* __restrict__ dsb) {
  __shared__ float red[3][4];
  float sl = 0.f, sg = 0.f, s0 = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) {
    sl += head == 0 ? (rlse[i] - diag[i]) + (clse[i] - diag[i]) : part[3 * i];
    sg += part[3 * i + 1];
    s0 += part[3 * i + 2];
  }
  sl = wave_sum(sl); sg = wave_sum(sg); s0 = wave_sum(s0);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sl; red[1][threadIdx.x >> 6] = sg; red[2][threadIdx.x >> 6] = s0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float L = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    loss[0] = head == 0 ? 0.5f * L / (float)n : L / (float)n;
    dsb[0] = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) / scale;
    dsb[1] = head == 0 ? 0.f : (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
  }
}

// out [cols_out, ld_out] = in [rows, cols]^T, zero-filled past `rows` up to
// ld_out columns.  32x32 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_pad(const float* __restrict__ in, int rows,
                                                       int cols, int ld_in,
                                                       float* __restrict__ out, int ld_out) {
  __shared__ float t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    t[k][tx] = (r < rows && c < cols) ? in[(size_t)r * ld_in + c] : 0.f;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;   // out row c, column r
    if (c < cols && r < ld_out) out[(size_t)c * ld_out + r] = t[tx][k];
  }
}

static hipError_t transpose_pad(const float* in, int rows, int cols, int ld_in, float* out,
                                int ld_out, hipStream_t s) {
  dim3 grid((cols + 31) / 32, (ld_out + 31) / 32), block(256);
  hipLaunchKernelGGL(k_transpose_pad, grid, block, 0, s, in, rows, cols, ld_in, out, ld_out);
  return hipGetLastError();
}

size_t contrastive_workspace_bytes(int n, int dim) {
  const size_t n16 = (size_t)(n + 15) / 16 * 16;
  auto a = [](size_t b) { return (b + 255) / 256 * 256; };
  return a(4 * (size_t)n * n16) * 2 + a(4 * (size_t)dim * n16) * 2 + a(4 * (size_t)n) * 3 +
         a(12 * (size_t)n);
}

hipError_t contrastive_loss(const float* E, const float* Tx, int n, int dim, int head,
                            float scale, float bias, float* loss, float* dE, float* dT,
                            float* dsb, void* ws, hipStream_t s) {
  const int n16 = (n + 15) / 16 * 16;
  auto a = [](size_t b) { return (b + 255) / 256 * 256; };
  char* w = static_cast<char*>(ws);
  float* L = reinterpret_cast<float*>(w);                 w += a(4 * (size_t)n * n16);
  float* Gt = reinterpret_cast<float*>(w);                w += a(4 * (size_t)n * n16);
  float* Tt = reinterpret_cast<float*>(w);                w += a(4 * (size_t)dim * n16);
  float* Et = reinterpret_cast<float*>(w);                w += a(4 * (size_t)dim * n16);
  float* rlse = reinterpret_cast<float*>(w);              w += a(4 * (size_t)n);
  float* clse = reinterpret_cast<float*>(w);              w += a(4 * (size_t)n);
  float* diag = reinterpret_cast<float*>(w);              w += a(4 * (size_t)n);
  float* part = reinterpret_cast<float*>(w);
  hipError_t err;
  // logits [n, n16] (the GEMM writes whole 4-column groups, so up to three
  // columns past n; every reader stops at n, and the gradient kernel zeroes
  // the padding)
  EpiArgs e;
  e.out = L; e.ldo = n16; e.alpha = scale; e.beta = bias;
  if ((err = gemm_f32(E, dim, Tx, dim, n, n, dim, OP_LOGITS, e, s)) != hipSuccess) return err;
  hipLaunchKernelGGL(k_row_lse, dim3(n), dim3(256), 0, s, L, n, n16, rlse);
  hipLaunchKernelGGL(k_col_lse, dim3((n + 63) / 64), dim3(256), 0, s, L, n, n16, clse);
  hipLaunchKernelGGL(k_diag, dim3((n + 255) / 256), dim3(256), 0, s, L, n, n16, diag);
  hipLaunchKernelGGL(k_contrastive_grad, dim3(n), dim3(256), 0, s, L, n, n16, head, bias, rlse,
                     clse, part);
  hipLaunchKernelGGL(k_contrastive_reduce, dim3(1), dim3(256), 0, s, part, rlse, clse, diag, n,
                     head, scale, loss, dsb);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  // dE = scale * G T : A = G [n, n16], B = T^T [dim, n16]
  if ((err = transpose_pad(Tx, n, dim, dim, Tt, n16, s)) != hipSuccess) return err;
  EpiArgs ge;
  ge.out = dE; ge.ldo = dim; ge.alpha = scale; ge.beta = 0.f;
  if ((err = gemm_f32(L, n16, Tt, n16, n, dim, n16, OP_LOGITS, ge, s)) != hipSuccess) return err;
  // dT = scale * G^T E : A = G^T [n, n16], B = E^T [dim, n16]
  if ((err = transpose_pad(L, n, n, n16, Gt, n16, s)) != hipSuccess) return err;
  if ((err = transpose_pad(E, n, dim, dim, Et, n16, s)) != hipSuccess) return err;
  EpiArgs gt;
  gt.out = dT; gt.ldo = dim; gt.alpha = scale; gt.beta = 0.f;
  return gemm_f32(Gt, n16, Et, n16, n, dim, n16, OP_LOGITS, gt, s);
}

// Scratch of the allocation-free contrastive entry point: a file-scope
// device array, one copy per GPU, alive until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); it asks the runtime for the array's device
// address once per device, with that device current, and uses that address.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace vl
