// PCG vector kernels (Algorithm 2 step 4): scaled copies, dot products with
// two-stage deterministic reductions, and the fused y/r and p updates. The
// step scalars (alpha, beta, rho) stay in device memory so that one PCG
// iteration needs a single device-to-host read (the stopping norm).
#include "common.h"

namespace lsq {

constexpr int kVecThreads = 256;
constexpr int kMaxPartials = 1024;

static int vec_blocks(int64_t n) {
  int64_t b = (n + kVecThreads * 4 - 1) / (kVecThreads * 4);
  if (b < 1) b = 1;
  if (b > kMaxPartials) b = kMaxPartials;
  return (int)b;
}

template <typename T>
__global__ void k_scale(int64_t n, const T *__restrict__ a, const T *__restrict__ x, T *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] * x[i];
}

template <typename T>
__global__ void k_copy(int64_t n, const T *__restrict__ x, T *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

__device__ __forceinline__ void finish_op(double *scal, int dst, int op, double acc) {
  {
    if (op == 0) {
      scal[dst] = acc;
    } else if (op == 1) {  // p.q -> alpha = rho / (p.q)
      scal[Scal::PQ] = acc;
      scal[Scal::ALPHA] = scal[Scal::RHO] / acc;
    } else if (op == 2) {  // r.z at a (re)start: rho = rho_new = r.z
      scal[Scal::RHO] = acc;
      scal[Scal::RHO_NEW] = acc;
    } else {  // r.z in a later iteration: beta = rho_new / rho, then rho = rho_new
      scal[Scal::RHO_NEW] = acc;
      scal[Scal::BETA] = acc / scal[Scal::RHO];
      scal[Scal::RHO] = acc;
    }
  }
}

// after part[blockIdx.x] is written: the last workgroup to arrive sums the
// partials exactly as k_finish does (same thread layout and order) and
// applies the op, then clears the count for the next reduction
__device__ __forceinline__ void finish_if_last(const double *part, const Fin &fin) {
  __shared__ double red[kVecThreads / kWave];
  __shared__ bool last;
  __syncthreads();  // thread 0 has written this workgroup's partial
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(fin.cnt, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double acc = 0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x)
    acc += __hip_atomic_load(part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    finish_op(fin.scal, fin.dst, fin.op, acc);
    __hip_atomic_store(fin.cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// partial sums of x.*y, or of (d.*x)^2 when y is null
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_dot_part(int64_t n, const T *__restrict__ x,
                                                          const T *__restrict__ y,
                                                          const double *__restrict__ d,
                                                          double *__restrict__ part, Fin fin) {
  __shared__ T red[kVecThreads / kWave];
  T acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (y) {
      acc += x[i] * y[i];
    } else {
      T v = d ? (T)d[i] * x[i] : x[i];
      acc += v * v;
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = (double)acc;
  if (fin.cnt) finish_if_last(part, fin);
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_update_yr(int64_t n, const double *__restrict__ alpha,
                                                           const T *__restrict__ p, const T *__restrict__ q,
                                                           T *__restrict__ y, T *__restrict__ r,
                                                           const double *__restrict__ d,
                                                           double *__restrict__ part, Fin fin) {
  __shared__ T red[kVecThreads / kWave];
  const T a = (T)(*alpha);
  T acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    y[i] += a * p[i];
    T ri = r[i] - a * q[i];
    r[i] = ri;
    T v = d ? (T)d[i] * ri : ri;
    acc += v * v;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = (double)acc;
  if (fin.cnt) finish_if_last(part, fin);
}

template <typename T>
__global__ void k_update_p(int64_t n, const double *__restrict__ beta, const T *__restrict__ z,
                           T *__restrict__ p) {
  const T bt = beta ? (T)(*beta) : (T)0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = beta ? z[i] + bt * p[i] : z[i];
}

// p = z + beta p (p = z without beta) and u = s p, the scaled input of the
// next operator product
template <typename T>
__global__ void k_update_p_scaled(int64_t n, const double *__restrict__ beta, const T *__restrict__ z,
                                  T *__restrict__ p, const T *__restrict__ s, T *__restrict__ u) {
  const T bt = beta ? (T)(*beta) : (T)0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T pi = beta ? z[i] + bt * p[i] : z[i];
    p[i] = pi;
    u[i] = s[i] * pi;
  }
}

__global__ __launch_bounds__(256) void k_finish(const double *__restrict__ part, int np, double *scal, int dst,
                                                int op) {
  __shared__ double red[256 / kWave];
  double acc = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) finish_op(scal, dst, op, acc);
}


__global__ void k_axpy_scaled(int64_t n, double nu, const double *__restrict__ invD, const float *__restrict__ d,
                              double *__restrict__ x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += invD[i] * (nu * (double)d[i]);
}

__global__ void k_f64_to_f32_scaled(int64_t n, const double *__restrict__ x, const double *__restrict__ s,
                                    double mul, float *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)((s ? s[i] * x[i] : x[i]) * mul);
}

__global__ void k_widen(int64_t n, const float *__restrict__ x, double *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

__global__ void k_sub(int64_t n, const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] - b[i];
}

static dim3 grid_for(int64_t n) {
  int64_t b = (n + kVecThreads - 1) / kVecThreads;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

template <typename T>
void Vec<T>::scale(int64_t n, const T *a, const T *x, T *y, hipStream_t st) {
  k_scale<T><<<grid_for(n), kVecThreads, 0, st>>>(n, a, x, y);
}
template <typename T>
void Vec<T>::copy(int64_t n, const T *x, T *y, hipStream_t st) {
  k_copy<T><<<grid_for(n), kVecThreads, 0, st>>>(n, x, y);
}
template <typename T>
int Vec<T>::dot_partials(int64_t n, const T *x, const T *y, const double *d, double *part, hipStream_t st,
                         const Fin *fin) {
  int nb = vec_blocks(n);
  k_dot_part<T><<<nb, kVecThreads, 0, st>>>(n, x, y, d, part, fin ? *fin : Fin{});
  return nb;
}
template <typename T>
int Vec<T>::update_yr(int64_t n, const double *alpha, const T *p, const T *q, T *y, T *r, const double *d,
                      double *part, hipStream_t st, const Fin *fin) {
  int nb = vec_blocks(n);
  k_update_yr<T><<<nb, kVecThreads, 0, st>>>(n, alpha, p, q, y, r, d, part, fin ? *fin : Fin{});
  return nb;
}
template <typename T>
void Vec<T>::update_p(int64_t n, const double *beta, const T *z, T *p, hipStream_t st) {
  k_update_p<T><<<grid_for(n), kVecThreads, 0, st>>>(n, beta, z, p);
}

template <typename T>
void Vec<T>::update_p_scaled(int64_t n, const double *beta, const T *z, T *p, const T *s, T *u, hipStream_t st) {
  k_update_p_scaled<T><<<grid_for(n), kVecThreads, 0, st>>>(n, beta, z, p, s, u);
}

template struct Vec<double>;
template struct Vec<float>;

void launch_finish(const double *part, int np, double *scal, int dst, int op, hipStream_t st) {
  k_finish<<<1, 256, 0, st>>>(part, np, scal, dst, op);
}
void launch_axpy_scaled_f64(int64_t n, double nu, const double *invD, const float *d, double *x, hipStream_t st) {
  k_axpy_scaled<<<grid_for(n), kVecThreads, 0, st>>>(n, nu, invD, d, x);
}
void launch_f64_to_f32_scaled(int64_t n, const double *x, const double *s, double mul, float *y, hipStream_t st) {
  k_f64_to_f32_scaled<<<grid_for(n), kVecThreads, 0, st>>>(n, x, s, mul, y);
}
void launch_f32_to_f64(int64_t n, const float *x, double *y, hipStream_t st) {
  k_widen<<<grid_for(n), kVecThreads, 0, st>>>(n, x, y);
}
void launch_sub_f64(int64_t n, const double *a, const double *b, double *y, hipStream_t st) {
  k_sub<<<grid_for(n), kVecThreads, 0, st>>>(n, a, b, y);
}

}  // namespace lsq
