// Small device utilities: operator upload (column-major -> row-major), row-sum
// infinity norms, FN evaluation at arbitrary points.
#include "engine.hpp"

namespace nep {

// out[r*n + c] = in[r + c*ld]  (real or complex elements of `words` doubles)
__global__ void k_to_rowmajor(const double* __restrict__ in, long long ld, int n, int words,
                              double* __restrict__ out) {
  __shared__ double tile[32][33 * 2];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx: column block, by: row block
  const int tx = threadIdx.x, ty = threadIdx.y;          // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int c = bx + k, r = by + tx;
    if (r < n && c < n)
      for (int w = 0; w < words; ++w) tile[k][tx * words + w] = in[(r + c * ld) * words + w];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int r = by + k, c = bx + tx;
    if (r < n && c < n)
      for (int w = 0; w < words; ++w) out[((long long)r * n + c) * words + w] = tile[tx][k * words + w];
  }
}

hipError_t to_rowmajor(const void* in, long long ld, int n, int cplx, void* out, hipStream_t st) {
  dim3 grid(ceil_div(n, 32), ceil_div(n, 32)), blk(32, 8);
  hipLaunchKernelGGL(k_to_rowmajor, grid, blk, 0, st, (const double*)in, ld, n, cplx ? 2 : 1, (double*)out);
  return hipGetLastError();
}

// ||A||_inf = max_r sum_c |a_rc| of a row-major matrix; one block per row chunk.
__global__ void k_inf_norm(const double* __restrict__ A, int n, int cplx, unsigned long long* __restrict__ out) {
  __shared__ double red[256];
  double best = 0.0;
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    double s = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      if (cplx) {
        const double re = A[2 * ((long long)r * n + c)], im = A[2 * ((long long)r * n + c) + 1];
        s += sqrt(re * re + im * im);
      } else {
        s += fabs(A[(long long)r * n + c]);
      }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) best = fmax(best, red[0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(best));
}

__global__ void k_bits_to_double(const unsigned long long* __restrict__ in, double* __restrict__ out, int cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) out[i] = __longlong_as_double((long long)in[i]);
}

hipError_t inf_norm(const void* A, int n, int cplx, unsigned long long* scratch, double* out, hipStream_t st) {
  hipError_t e = hipMemsetAsync(scratch, 0, sizeof(unsigned long long), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_inf_norm, dim3(std::min(n, 1024)), dim3(256), 0, st, (const double*)A, n, cplx, scratch);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bits_to_double, dim3(1), dim3(64), 0, st, scratch, out, 1);
  return hipGetLastError();
}

// dst = src^* (conjugate transpose) of a row-major n x n matrix, real or
// complex, through 32 x 32 LDS tiles.
__global__ void k_adjoint_copy(const double* __restrict__ src, int n, int cplx, double* __restrict__ dst) {
  __shared__ double tre[32][33], tim[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = by + k, c = bx + threadIdx.x;
    if (r < n && c < n) {
      const long long e = (long long)r * n + c;
      tre[k][threadIdx.x] = cplx ? src[2 * e] : src[e];
      tim[k][threadIdx.x] = cplx ? src[2 * e + 1] : 0.0;
    }
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = bx + k, c = by + threadIdx.x;  // dst[r][c] = conj(src[c][r])
    if (r < n && c < n) {
      const long long e = (long long)r * n + c;
      if (cplx) {
        dst[2 * e] = tre[threadIdx.x][k];
        dst[2 * e + 1] = -tim[threadIdx.x][k];
      } else {
        dst[e] = tre[threadIdx.x][k];
      }
    }
  }
}

hipError_t adjoint_copy(const void* src, int n, int cplx, void* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint_copy, dim3(ceil_div(n, 32), ceil_div(n, 32)), dim3(32, 8), 0, st,
                     static_cast<const double*>(src), n, cplx, static_cast<double*>(dst));
  return hipGetLastError();
}

__global__ void k_conj_copy(const c128* __restrict__ src, int n, c128* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = conj(src[i]);
}

hipError_t conj_copy(const c128* src, int n, c128* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_conj_copy, dim3(ceil_div(n, 256)), dim3(256), 0, st, src, n, dst);
  return hipGetLastError();
}

// f_i(z_k) for k < m, i < ell; out[i*m + k]; bad flags per point.
__global__ void k_fn_points(const FnNode* __restrict__ nodes, const c128* __restrict__ coef, const int* __restrict__ roots,
                            int ell, const c128* __restrict__ z, int m, c128* __restrict__ out, int* __restrict__ bad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  int b = 0;
  for (int i = 0; i < ell; ++i) out[(long long)i * m + k] = fn_eval(nodes, coef, roots[i], z[k], b);
  bad[k] = b;
}

hipError_t fn_points(const FnNode* nodes, const c128* coef, const int* roots, int ell, const c128* z, int m,
                     c128* out, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_fn_points, dim3(ceil_div(m, 64)), dim3(64), 0, st, nodes, coef, roots, ell, z, m, out, bad);
  return hipGetLastError();
}

// f_i'(z_k): out[i*m + k].
__global__ void k_fn_points_d(const FnNode* __restrict__ nodes, const c128* __restrict__ coef,
                              const int* __restrict__ roots, int ell, const c128* __restrict__ z, int m,
                              c128* __restrict__ out, int* __restrict__ bad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  int b = 0;
  for (int i = 0; i < ell; ++i) {
    c128 d;
    (void)fn_eval_d(nodes, coef, roots[i], z[k], b, d);
    out[(long long)i * m + k] = d;
  }
  bad[k] = b;
}

hipError_t fn_points_d(const FnNode* nodes, const c128* coef, const int* roots, int ell, const c128* z, int m,
                       c128* out, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_fn_points_d, dim3(ceil_div(m, 64)), dim3(64), 0, st, nodes, coef, roots, ell, z, m, out, bad);
  return hipGetLastError();
}

}  // namespace nep
