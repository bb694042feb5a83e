// Support kernels of the hybrid step: fills, pass set-up (fixed-point units
// from device-resident bounds), tally decoding, the remap source (step 3 of
// Sec. 2.2), deterministic prefix scans, and census population control.
#include "slh_common.hpp"

namespace slh {

// ---------------------------------------------------------------------------
// fills (kernels rather than hipMemset so that a captured graph replays them)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, long long n, T v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
static hipError_t fill(T* p, long long n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 4096 ? b : 4096);
  hipLaunchKernelGGL(k_fill<T>, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, long long n, unsigned long long v,
                           hipStream_t s) { return fill(p, n, v, s); }
hipError_t launch_fill_u8(uint8_t* p, long long n, uint8_t v, hipStream_t s) {
  return fill(p, n, v, s);
}
hipError_t launch_fill_f64(double* p, long long n, double v, hipStream_t s) {
  return fill(p, n, v, s);
}

// ---------------------------------------------------------------------------
// Pass set-up.  Bounds: |w| of a source particle <= sum(M)/N_p, so the
// source weight magnitude is <= sum(M); census-in magnitude <= n_in max|w|.
// Weights only decay along a path and a path lasts at most c dt, so every
// balance sum is <= W and every tally sum is <= W c dt.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void unit_for(double bound, double& unit, double& inv) {
  if (!(bound > 0.0)) { unit = 1.0; inv = 1.0; return; }
  int e;
  frexp(bound, &e);  // bound < 2^e
  unit = ldexp(1.0, e - 61);
  inv = ldexp(1.0, 61 - e);
}

__global__ void k_pass_begin(DevState* st, const double* cdf, long long n_cells, double cdt) {
  const int t = threadIdx.x;
  if (t < 2 * B_NFIELDS) st->bal[t] = 0ull;
  if (t == 0) {
    const double total = n_cells > 0 ? cdf[n_cells - 1] : 0.0;
    const double W = (double)st->n_in * st->maxabs_w + total;
    unit_for(W, st->unit_W, st->inv_W);
    unit_for(W * cdt, st->unit_T, st->inv_T);
    st->work = 0ull;
    st->segments = 0ull;
    st->particles = 0ull;
    st->killed = 0ull;
    st->alive = 0ull;
  }
}

hipError_t launch_pass_begin(DevState* st, const double* cdf, long long n_cells, double cdt,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(64), 0, s, st, cdf, n_cells, cdt);
  return hipGetLastError();
}

__global__ void k_tally_to_flux(const unsigned long long* __restrict__ T, long long n,
                                const DevState* st, double inv_adt, double* __restrict__ phi) {
  const double unit = st->unit_T;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    phi[i] = fix_value((long long)T[2 * i], (long long)T[2 * i + 1], unit) * inv_adt;
}

hipError_t launch_tally_to_flux(const unsigned long long* T, long long n, const DevState* st,
                                double inv_adt, double* phi, hipStream_t s) {
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
  hipLaunchKernelGGL(k_tally_to_flux, dim3(grid), dim3(256), 0, s, T, n, st, inv_adt, phi);
  return hipGetLastError();
}

// q_R = Q + sigma_s (phi_pre + phi_post) + sigma_s phi_c (nodal, bilinear);
// majorant M = A dt max_corner |q_R|.
__global__ void k_remap_source(long long n, const double* __restrict__ q,
                               const double* __restrict__ sig_s,
                               const double* __restrict__ phi_pre,
                               const double* __restrict__ phi_post,
                               const double* __restrict__ phi_c, double adt,
                               double* __restrict__ qn, double* __restrict__ M) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double ss = sig_s[i];
    const double base = q[i] + ss * (phi_pre[i] + phi_post[i]);
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double v = base + ss * phi_c[4 * i + k];
      qn[4 * i + k] = v;
      mx = fmax(mx, fabs(v));
    }
    M[i] = adt * mx;
  }
}

hipError_t launch_remap_source(long long n, const double* q, const double* sig_s,
                               const double* phi_pre, const double* phi_post,
                               const double* phi_c, double adt, double* qn, double* M,
                               hipStream_t s) {
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
  hipLaunchKernelGGL(k_remap_source, dim3(grid), dim3(256), 0, s, n, q, sig_s, phi_pre,
                     phi_post, phi_c, adt, qn, M);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inclusive prefix scan, fixed association order (deterministic): blocks of
// 1024 elements (4 per thread), recursive scan of block totals, add-back.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_block(const T* in, T* out, long long n,
                                                             T* sums) {
  __shared__ T s[kScanThreads];
  const long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanPer;
  T v[kScanPer];
  T run = T(0);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const long long i = base + k;
    run = run + (i < n ? in[i] : T(0));
    v[k] = run;
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const T add = (int)threadIdx.x >= off ? s[threadIdx.x - off] : T(0);
    __syncthreads();
    s[threadIdx.x] = s[threadIdx.x] + add;
    __syncthreads();
  }
  const T before = threadIdx.x > 0 ? s[threadIdx.x - 1] : T(0);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const long long i = base + k;
    if (i < n) out[i] = before + v[k];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s[threadIdx.x];
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_add(T* out, long long n, const T* sums) {
  const long long blk = blockIdx.x + 1;  // block 0 needs nothing
  const T add = sums[blk - 1];
  for (int k = threadIdx.x; k < kScanBlock; k += kScanThreads) {
    const long long i = blk * kScanBlock + k;
    if (i < n) out[i] = out[i] + add;
  }
}

size_t scan_tmp_elems(long long n) {
  size_t tot = 0;
  while (n > 1) {
    n = (n + kScanBlock - 1) / kScanBlock;
    tot += (size_t)n + 1;
  }
  return tot + 1;
}

template <typename T>
static hipError_t scan_rec(const T* in, T* out, long long n, T* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_block<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                     tmp);
  if (nb > 1) {
    hipError_t e = scan_rec<T>(tmp, tmp, nb, tmp + nb + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)(nb - 1)), dim3(kScanThreads), 0, s, out,
                       n, (const T*)tmp);
  }
  return hipGetLastError();
}

hipError_t scan_inclusive_f64(const double* in, double* out, long long n, double* tmp,
                              hipStream_t s) { return scan_rec<double>(in, out, n, tmp, s); }
hipError_t scan_inclusive_i64(const long long* in, long long* out, long long n,
                              long long* tmp, hipStream_t s) {
  return scan_rec<long long>(in, out, n, tmp, s);
}

// ---------------------------------------------------------------------------
// Census population control: when more than `cap` particles reach t_{n+1},
// keep the cap particles with the smallest thinning keys
// key = mix64(thin_stream ^ hid) (a bijection of the unique history ids, so
// keys are distinct: a simple random sample without replacement) and scale
// their weights by count/cap.  The cap-th smallest key is found by an 8-pass
// radix select on 8-bit digits with integer histograms.
// ---------------------------------------------------------------------------
__global__ void k_select_init(DevState* st, long long cap) {
  if (threadIdx.x != 0) return;
  const unsigned long long cnt = st->alive;
  st->thin_active = cnt > (unsigned long long)cap ? 1 : 0;
  st->thin_factor = st->thin_active ? (double)cnt / (double)cap : 1.0;
  st->sel_prefix = 0ull;
  st->sel_rank = cap > 0 ? (unsigned long long)(cap - 1) : 0ull;
  st->maxabs_bits_out = 0ull;
}

__global__ __launch_bounds__(256) void k_select_hist(const uint8_t* __restrict__ alive,
                                                     const uint64_t* __restrict__ hid,
                                                     long long n, uint64_t thin_stream,
                                                     const DevState* st, int shift,
                                                     unsigned long long* hist) {
  if (!st->thin_active) return;
  __shared__ unsigned int s_h[256];
  s_h[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned long long prefix = st->sel_prefix;
  const int high = shift + 8;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    if (!alive[i]) continue;
    const unsigned long long key = mix64(thin_stream ^ hid[i]);
    if (high < 64 && (key >> high) != (prefix >> high)) continue;
    atomicAdd(&s_h[(key >> shift) & 255ull], 1u);
  }
  __syncthreads();
  if (s_h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)s_h[threadIdx.x]);
}

__global__ void k_select_pick(DevState* st, unsigned long long* hist, int shift) {
  if (threadIdx.x != 0) return;
  if (st->thin_active) {
    unsigned long long rank = st->sel_rank, cum = 0ull;
    for (int b = 0; b < 256; ++b) {
      if (cum + hist[b] > rank) {
        st->sel_prefix |= (unsigned long long)b << shift;
        st->sel_rank = rank - cum;
        break;
      }
      cum += hist[b];
    }
  }
  for (int b = 0; b < 256; ++b) hist[b] = 0ull;
}

hipError_t launch_census_select(const uint8_t* alive, const uint64_t* hid, long long n,
                                long long cap, uint64_t thin_stream, DevState* st,
                                unsigned long long* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_select_init, dim3(1), dim3(1), 0, s, st, cap);
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    hipLaunchKernelGGL(k_select_hist, dim3(grid), dim3(256), 0, s, alive, hid, n, thin_stream,
                       (const DevState*)st, shift, hist);
    hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(1), 0, s, st, hist, shift);
  }
  return hipGetLastError();
}

__global__ void k_census_flags(const uint8_t* __restrict__ alive,
                               const uint64_t* __restrict__ hid, long long n,
                               uint64_t thin_stream, const DevState* st,
                               long long* __restrict__ flags) {
  const int act = st->thin_active;
  const unsigned long long kmax = st->sel_prefix;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    long long f = alive[i] ? 1 : 0;
    if (f && act) f = mix64(thin_stream ^ hid[i]) <= kmax ? 1 : 0;
    flags[i] = f;
  }
}

hipError_t launch_census_flags(const uint8_t* alive, const uint64_t* hid, long long n,
                               uint64_t thin_stream, const DevState* st, long long* flags,
                               hipStream_t s) {
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
  hipLaunchKernelGGL(k_census_flags, dim3(grid), dim3(256), 0, s, alive, hid, n, thin_stream,
                     st, flags);
  return hipGetLastError();
}

template <typename R>
__global__ void k_census_compact(Bank<R> src, const long long* __restrict__ incl, long long n,
                                 Bank<R> dst, DevState* st) {
  const R f = (R)st->thin_factor;
  double mx = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long before = i > 0 ? incl[i - 1] : 0;
    if (incl[i] == before) continue;
    const long long d = before;
    dst.px[d] = src.px[i];
    dst.py[d] = src.py[i];
    dst.ox[d] = src.ox[i];
    dst.oy[d] = src.oy[i];
    const R w = src.w[i] * f;
    dst.w[d] = w;
    dst.cell[d] = src.cell[i];
    dst.hid[d] = src.hid[i];
    mx = fmax(mx, fabs((double)w));
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if (__lane_id() == 0 && mx > 0.0)
    atomicMax(&st->maxabs_bits_out, (unsigned long long)__double_as_longlong(mx));
}

template <typename R>
hipError_t launch_census_compact(const Bank<R>& src, const long long* incl, long long n,
                                 Bank<R> dst, DevState* st, hipStream_t s) {
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
  hipLaunchKernelGGL(k_census_compact<R>, dim3(grid), dim3(256), 0, s, src, incl, n, dst, st);
  return hipGetLastError();
}
template hipError_t launch_census_compact<double>(const Bank<double>&, const long long*,
                                                  long long, Bank<double>, DevState*,
                                                  hipStream_t);
template hipError_t launch_census_compact<float>(const Bank<float>&, const long long*,
                                                 long long, Bank<float>, DevState*,
                                                 hipStream_t);

__global__ void k_census_finish(DevState* st, const long long* incl, long long n) {
  if (threadIdx.x != 0) return;
  st->n_in = n > 0 ? incl[n - 1] : 0;
  st->n_kept = st->n_in;
  st->maxabs_w = __longlong_as_double((long long)st->maxabs_bits_out);
}

hipError_t launch_census_finish(DevState* st, const long long* incl, long long n,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_census_finish, dim3(1), dim3(1), 0, s, st, incl, n);
  return hipGetLastError();
}

}  // namespace slh
