// Support kernels of the hybrid step: fills, pass set-up (fixed-point units
// from device-resident bounds), tally decoding, the remap source (step 3 of
// Sec. 2.2), deterministic prefix scans, and census population control.
#include <algorithm>

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
// Pass set-up.  Bounds: |w| of a source particle <= w_q, so the source weight
// magnitude is <= (particles) w_q; census-in magnitude <= n_in max|w|.
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

// Pass set-up fused with the clears the pass needs: block 0 resets the
// pass counters and balance and sets the fixed-point units from the bounds;
// every block clears its share of up to two tally arrays and a byte array.
__global__ void k_pass_prep(DevState* st, const double* ctree, int kind, long long src_cap,
                            double cdt, unsigned long long* __restrict__ a, long long na,
                            unsigned long long* __restrict__ b, long long nb,
                            uint8_t* __restrict__ c, long long nc) {
  if (st->halt) return;
  if (blockIdx.x == 0) {
    const int t = threadIdx.x;
    if (t < 2 * B_NFIELDS) st->bal[t] = 0ull;
    if (t == 0) {
      const double n_emit = ctree[1];
      const bool over = !(n_emit <= (double)src_cap);
      const double src = (over ? (double)src_cap : n_emit) * st->wq[kind - 1];
      const double W = (double)st->n_in * st->maxabs_w + src;
      unit_for(W, st->unit_W, st->inv_W);
      unit_for(W * cdt, st->unit_T, st->inv_T);
      st->work = 0ull;
      st->segments = 0ull;
      st->particles = 0ull;
      st->killed = 0ull;
      st->alive = 0ull;
      st->n_emit = over ? src_cap : (long long)n_emit;
      st->numeric = (isfinite(st->sumM[kind - 1]) ? 0 : 1) | (over ? 4 : 0);
    }
  }
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long str = (long long)gridDim.x * blockDim.x;
  for (long long i = i0; i < na; i += str) a[i] = 0ull;
  for (long long i = i0; i < nb; i += str) b[i] = 0ull;
  for (long long i = i0; i < nc; i += str) c[i] = 0;
}

hipError_t launch_pass_prep(DevState* st, const double* ctree, int kind, long long src_cap,
                            double cdt, unsigned long long* a, long long na,
                            unsigned long long* b, long long nb, uint8_t* c, long long nc,
                            hipStream_t s) {
  long long n = na > nb ? na : nb;
  n = n > nc ? n : nc;
  long long g = (n + 255) / 256;
  const int grid = (int)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
  hipLaunchKernelGGL(k_pass_prep, dim3(grid), dim3(256), 0, s, st, ctree, kind, src_cap, cdt, a,
                     na, b, nb, c, nc);
  return hipGetLastError();
}

// phi = (sum of the private copies, an exact integer sum) * unit / (A dt).
// A block takes 64 cells; its four waves each sum every fourth copy (eight
// loads in flight per lane) and the four partial sums meet in LDS.  Integer
// addition makes the result independent of this split.
constexpr int kT2fCells = 64;
__global__ __launch_bounds__(256) void k_tally_to_flux(const unsigned long long* __restrict__ T0,
                                                       double* __restrict__ phi0,
                                                       const unsigned long long* __restrict__ T1,
                                                       double* __restrict__ phi1, long long n,
                                                       int n_copies, long long copy_stride,
                                                       const DevState* st, double inv_adt) {
  if (st->halt) return;
  // blockIdx.y picks one of two tallies decoded by the same launch
  const unsigned long long* __restrict__ T = blockIdx.y ? T1 : T0;
  double* __restrict__ phi = blockIdx.y ? phi1 : phi0;
  __shared__ unsigned long long s_part[4][kT2fCells];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long i = (long long)blockIdx.x * kT2fCells + lane;
  const long long ic = i < n ? i : n - 1;  // a real cell for every lane's loads
  const unsigned long long* p = T + kTallyStride * ic;
  unsigned long long v = 0ull;
  int c = w;
  for (; c + 28 < n_copies; c += 32) {
    unsigned long long t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p[(long long)(c + 4 * u) * copy_stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; c < n_copies; c += 4) v += p[(long long)c * copy_stride];
  s_part[w][lane] = v;
  __syncthreads();
  if (w == 0 && i < n) {
    const unsigned long long s = s_part[0][lane] + s_part[1][lane] + s_part[2][lane] + s_part[3][lane];
    phi[i] = (double)(long long)s * st->unit_T * inv_adt;
  }
}

hipError_t launch_tally_to_flux(const unsigned long long* T0, double* phi0,
                                const unsigned long long* T1, double* phi1, long long n,
                                int n_copies, long long copy_stride, const DevState* st,
                                double inv_adt, hipStream_t s) {
  if (n < 1) return hipSuccess;
  const long long b = (n + kT2fCells - 1) / kT2fCells;
  if (b > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tally_to_flux, dim3((unsigned)b, T1 ? 2 : 1), dim3(256), 0, s, T0, phi0,
                     T1, phi1, n, n_copies, copy_stride, st, inv_adt);
  return hipGetLastError();
}

// q_R = Q + sigma_s (phi_pre + phi_post) + sigma_s phi_c (nodal, bilinear).
__global__ void k_remap_source(long long n, const double* __restrict__ q,
                               const double* __restrict__ sig_s,
                               const double* __restrict__ phi_pre,
                               const double* __restrict__ phi_post,
                               const double* __restrict__ phi_c, double* __restrict__ qn,
                               const int* halt) {
  if (*halt) return;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double ss = sig_s[i];
    const double base = q[i] + ss * (phi_pre[i] + phi_post[i]);
    const double4 c = reinterpret_cast<const double4*>(phi_c)[i];
    reinterpret_cast<double4*>(qn)[i] =
        make_double4(base + ss * c.x, base + ss * c.y, base + ss * c.z, base + ss * c.w);
  }
}

hipError_t launch_remap_source(long long n, const double* q, const double* sig_s,
                               const double* phi_pre, const double* phi_post,
                               const double* phi_c, double* qn, const int* halt,
                               hipStream_t s) {
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
  hipLaunchKernelGGL(k_remap_source, dim3(grid), dim3(256), 0, s, n, q, sig_s, phi_pre,
                     phi_post, phi_c, qn, halt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Emission plan of a pass.  The cell majorant is M_i = adt pow2_ceil(m_i),
// m_i the largest corner |q_i|, so M_i takes one of the values
// V_b = adt 2^(b - 1074), b = 0 .. kMajBins - 1, and sum(M) = sum_b c_b V_b
// with c_b the number of cells in bin b.  The histogram is exact (integer
// counts), and the sum is formed exactly as an integer multiple of 2^-1074 in
// a multi-word accumulator and rounded once to the nearest double (ties to
// even): the correctly rounded sum of the majorants, whatever the order of
// the cells.  The counts are then n_i = floor(r_i) + [u_i < frac(r_i)],
// r_i = M_i / w_q, and their sum tree gives every particle its cell.
// ---------------------------------------------------------------------------
long long tree_leaves(long long n_cells) {
  long long L = 1;
  while (L < n_cells) L *= 2;
  return L;
}

__device__ __forceinline__ double cell_majorant_pow2(const double4 q) {
  return pow2_ceil(fmax(fmax(fabs(q.x), fabs(q.y)), fmax(fabs(q.z), fabs(q.w))));
}

// bin of a power of two p = 2^(e - 1) (frexp(p) = (1/2, e)): b = e + 1073,
// from 0 (2^-1074) to 2097 (2^1023); the last bin holds non-finite values
constexpr int kMajBad = kMajBins - 1;
__device__ __forceinline__ int maj_bin(double p) {
  if (!isfinite(p)) return kMajBad;
  int e;
  frexp(p, &e);
  const int b = e + 1073;
  return b < 0 ? 0 : (b >= kMajBad ? kMajBad : b);
}

// Block histogram in LDS, then one global add per non-empty bin and block.
__global__ __launch_bounds__(256) void k_maj_hist(const double* __restrict__ qn, long long n,
                                                  unsigned long long* __restrict__ hist,
                                                  const int* halt) {
  if (*halt) return;
  __shared__ unsigned int s_h[kMajBins];
  for (int k = threadIdx.x; k < kMajBins; k += blockDim.x) s_h[k] = 0u;
  __syncthreads();
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double p = cell_majorant_pow2(reinterpret_cast<const double4*>(qn)[i]);
    if (p > 0.0) atomicAdd(&s_h[maj_bin(p)], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kMajBins; k += blockDim.x)
    if (s_h[k]) atomicAdd(&hist[k], (unsigned long long)s_h[k]);
}

// The faces of an inflow: one global add per face to the x-face (group 1)
// or y-face (group 2) histogram.
__global__ void k_face_hist(Emitters em, unsigned long long* __restrict__ hist, const int* halt) {
  if (*halt) return;
  for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < em.n_faces;
       f += (long long)gridDim.x * blockDim.x) {
    int k;
    const int side = face_side((int)f, em.nx, em.ny, &k);
    const double p = pow2_ceil(fabs(em.inflow[f]));
    if (p > 0.0) atomicAdd(&hist[(side < 2 ? 1 : 2) * kMajBins + maj_bin(p)], 1ull);
  }
}

constexpr int kSumLimbs = 36;  // 2304 bits above 2^-1074

// Bits [r, r + 64) of the 128-bit value (hi, lo), zero outside it.
__device__ __forceinline__ unsigned long long bits128(unsigned long long lo, unsigned long long hi,
                                                      int r) {
  if (r <= -64 || r >= 128) return 0ull;
  if (r < 0) return lo << (-r);
  if (r == 0) return lo;
  if (r < 64) return (lo >> r) | (hi << (64 - r));
  if (r == 64) return hi;
  return hi >> (r - 64);
}

// bits [b, b + n) of the accumulator (n <= 64, b >= 0)
__device__ __forceinline__ unsigned long long limbs_bits(const unsigned long long* acc, int b,
                                                         int n) {
  const int w = b >> 6, sh = b & 63;
  unsigned long long v = acc[w] >> sh;
  if (sh && w + 1 < kSumLimbs) v |= acc[w + 1] << (64 - sh);
  return n == 64 ? v : (v & ((1ull << n) - 1ull));
}

// The exact sum of the histogram, rounded once; w_q; and the histogram
// cleared for the next plan.  The block copies and clears the histogram and
// lists its non-empty bins (in any order: the sum below is exact integer
// arithmetic); then one wave sums them.  Lane k < kSumLimbs owns 64-bit limb
// k of the sum (bit 0 = 2^-1074): every listed bin's term c_b mant_b 2^pos_b
// adds its bits that fall in the limb, and the limb counts its own
// overflows; lane 0 then propagates the carries and rounds.
constexpr int kMajSumThreads = 256;
__global__ __launch_bounds__(kMajSumThreads) void k_maj_sum(unsigned long long* __restrict__ hist,
                                                            double adt, double cx, double cy,
                                                            long long n_src, int kind,
                                                            DevState* st) {
  if (st->halt) return;
  __shared__ unsigned long long s_h[kMajGroups * kMajBins];
  __shared__ unsigned short s_list[kMajGroups * kMajBins];
  __shared__ unsigned long long s_limb[kSumLimbs], s_carry[kSumLimbs];
  __shared__ int s_n, s_bad, s_ovf;
  const int lane = threadIdx.x;
  if (lane == 0) {
    s_n = 0;
    s_bad = 0;
    s_ovf = 0;
  }
  __syncthreads();
  constexpr int kN = kMajGroups * kMajBins;
  constexpr int kPer = (kN + kMajSumThreads - 1) / kMajSumThreads;
  unsigned long long v[kPer];  // every load in flight before the first use
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = lane + j * kMajSumThreads;
    v[j] = k < kN ? hist[k] : 0ull;
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = lane + j * kMajSumThreads;
    if (k >= kN) continue;
    hist[k] = 0ull;
    s_h[k] = v[j];
    if (v[j]) {
      if (k % kMajBins == kMajBad) s_bad = 1;
      else s_list[atomicAdd(&s_n, 1)] = (unsigned short)k;
    }
  }
  __syncthreads();
  if (s_bad) {
    // a majorant overflowed: no emission (flagged by the pass set-up)
    if (lane == 0) {
      st->sumM[kind - 1] = __builtin_huge_val();
      st->wq[kind - 1] = 0.0;
    }
    return;
  }
  const int n_list = s_n;
  unsigned long long acc = 0ull, carry = 0ull;
  bool overflow = false;
  // every emitter group (cells, x faces, y faces): the value of each of its
  // majorants in bin b is its constant times 2^(b - 1074)
  for (int i = 0; lane < 64 && i < n_list && !overflow; ++i) {
    const int gb = s_list[i];
    const int g = gb / kMajBins, b = gb - g * kMajBins;
    const unsigned long long c = s_h[gb];  // the same in every lane
    const double V = (g == 0 ? adt : g == 1 ? cx : cy) * ldexp(1.0, b - 1074);
    if (!(V > 0.0)) continue;
    if (!isfinite(V)) {
      overflow = true;
      break;
    }
    int e;
    const double m = frexp(V, &e);  // V = m 2^e, m in [1/2, 1)
    unsigned long long mant = (unsigned long long)ldexp(m, 53);
    int pos = e - 53 + 1074;        // V = mant 2^(pos - 1074)
    if (pos < 0) {                  // subnormal V: its low bits are zero
      mant >>= -pos;
      pos = 0;
    }
    const unsigned long long lo = c * mant, hi = __umul64hi(c, mant);
    const unsigned long long add = bits128(lo, hi, 64 * lane - pos);
    acc += add;
    carry += acc < add ? 1ull : 0ull;
  }
  if (lane == 0 && overflow) s_ovf = 1;  // the same in every lane of the wave
  if (lane < kSumLimbs) {
    s_limb[lane] = acc;
    s_carry[lane] = carry;
  }
  __syncthreads();
  if (lane != 0) return;
  if (s_ovf) {
    st->sumM[kind - 1] = __builtin_huge_val();
    st->wq[kind - 1] = 0.0;
    return;
  }
  unsigned long long cin = 0ull;
  for (int k = 0; k < kSumLimbs; ++k) {  // carries of limb k go to limb k + 1
    const unsigned long long v = s_limb[k] + cin;
    cin = (v < cin ? 1ull : 0ull) + s_carry[k];
    s_limb[k] = v;
  }
  const unsigned long long* L = s_limb;
  int top = -1;
  for (int k = kSumLimbs - 1; k >= 0 && top < 0; --k)
    if (L[k]) top = 64 * k + 63 - __clzll((long long)L[k]);
  double sum = 0.0;
  if (top >= 0 && top < 53) {
    sum = ldexp((double)L[0], -1074);  // fewer than 53 bits: exact
  } else if (top >= 53) {
    unsigned long long mant = limbs_bits(L, top - 52, 53);
    const unsigned long long rnd = limbs_bits(L, top - 53, 1);
    bool sticky = false;
    const int below = top - 53;  // bits [0, below) decide a tie
    for (int k = 0; k < (below >> 6) && !sticky; ++k) sticky = L[k] != 0ull;
    if (!sticky && (below & 63)) sticky = limbs_bits(L, below & ~63, below & 63) != 0ull;
    int ex = top - 52 - 1074;
    if (rnd && (sticky || (mant & 1ull))) {
      mant += 1ull;
      if (mant == (1ull << 53)) { mant >>= 1; ex += 1; }
    }
    sum = ldexp((double)mant, ex);
  }
  st->sumM[kind - 1] = sum;
  st->wq[kind - 1] = (sum > 0.0 && isfinite(sum) && n_src > 0) ? quantum5(sum / (double)n_src)
                                                                : 0.0;
}

constexpr int kTreeChunk = 1024;

// Level of width W (nodes W..2W-1): block b sums nodes [W + b C, W + (b+1) C)
// with C = min(W, 1024) up through log2(C) levels.  Leaves are integers, so
// every sum is exact.
__global__ __launch_bounds__(512) void k_tree_up(double* t, long long W, const int* halt) {
  if (*halt) return;
  __shared__ double buf[2][kTreeChunk];
  const long long C = W < kTreeChunk ? W : kTreeChunk;
  const long long base = W + (long long)blockIdx.x * C;
  for (int j = threadIdx.x; j < C; j += blockDim.x) buf[0][j] = t[base + j];
  __syncthreads();
  long long width = W, cnt = C;
  long long first = (long long)blockIdx.x * C;  // offset of this block within the level
  int cur = 0;
  while (cnt > 1) {
    cnt >>= 1;
    width >>= 1;
    first >>= 1;
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
      const double v = buf[cur][2 * j] + buf[cur][2 * j + 1];
      buf[1 - cur][j] = v;
      t[width + first + j] = v;
    }
    cur = 1 - cur;
    __syncthreads();
  }
}

// All levels above the leaves, in launches of ten levels.
static void tree_up_all(double* tree, long long L, const int* halt, hipStream_t s) {
  long long W = L;
  while (W > 1) {
    const long long C = W < kTreeChunk ? W : kTreeChunk;
    hipLaunchKernelGGL(k_tree_up, dim3((unsigned)(W / C)), dim3(512), 0, s, tree, W, halt);
    W /= C;
  }
}

__global__ void k_count_leaves(const double* __restrict__ qn, long long n, Emitters em,
                               long long L, double adt, uint64_t seed, int points, int kind,
                               const DevState* __restrict__ st, double* __restrict__ ct) {
  if (st->halt) return;
  const double wq = st->wq[kind - 1];
  const uint64_t step = st->step;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < L;
       i += (long long)gridDim.x * blockDim.x) {
    double c = 0.0;
    if (i < n + em.n_faces && wq > 0.0) {
      double Mi;
      if (i < n) {
        Mi = adt * cell_majorant_pow2(reinterpret_cast<const double4*>(qn)[i]);
      } else {
        int k;
        const int side = face_side((int)(i - n), em.nx, em.ny, &k);
        Mi = (side < 2 ? em.cx : em.cy) * pow2_ceil(fabs(em.inflow[i - n]));
      }
      if (Mi > 0.0 && isfinite(Mi)) {
        const double r = Mi / wq;
        const double fl = floor(r);
        const uint64_t cs = stream_seed(seed, step, (uint32_t)kind, 3u, (uint64_t)i);
        const double u = u01_f64(point_u32_first(points, cs, 0u));
        c = fl + ((u < r - fl) ? 1.0 : 0.0);
      }
    }
    ct[L + i] = c;
  }
}

hipError_t launch_emission_plan(const double* qn, long long n_cells, const Emitters& em,
                                double adt, long long n_src, uint64_t seed, int points, int kind,
                                unsigned long long* hist, double* ctree, DevState* st,
                                hipStream_t s) {
  const long long L = tree_leaves(n_cells + em.n_faces);
  long long b = (n_cells + 255) / 256;
  int grid = (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
  const int* halt = &st->halt;
  hipLaunchKernelGGL(k_maj_hist, dim3(grid), dim3(256), 0, s, qn, n_cells, hist, halt);
  if (em.n_faces > 0)
    hipLaunchKernelGGL(k_face_hist, dim3((unsigned)((em.n_faces + 255) / 256)), dim3(256), 0, s,
                       em, hist, halt);
  hipLaunchKernelGGL(k_maj_sum, dim3(1), dim3(kMajSumThreads), 0, s, hist, adt, em.cx, em.cy, n_src, kind, st);
  b = (L + 255) / 256;
  grid = (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
  hipLaunchKernelGGL(k_count_leaves, dim3(grid), dim3(256), 0, s, qn, n_cells, em, L, adt, seed,
                     points, kind, (const DevState*)st, ctree);
  tree_up_all(ctree, L, halt, s);  // integer-valued sums below 2^53: exact
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
                                                             T* sums, const int* halt) {
  if (*halt) return;
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
__global__ __launch_bounds__(kScanThreads) void k_scan_add(T* out, long long n, const T* sums,
                                                           const int* halt) {
  if (*halt) return;
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
static hipError_t scan_rec(const T* in, T* out, long long n, T* tmp, const int* halt,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_block<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                     tmp, halt);
  if (nb > 1) {
    hipError_t e = scan_rec<T>(tmp, tmp, nb, tmp + nb + 1, halt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)(nb - 1)), dim3(kScanThreads), 0, s, out,
                       n, (const T*)tmp, halt);
  }
  return hipGetLastError();
}

hipError_t scan_inclusive_i64(const long long* in, long long* out, long long n,
                              long long* tmp, const int* halt, hipStream_t s) {
  return scan_rec<long long>(in, out, n, tmp, halt, s);
}

// ---------------------------------------------------------------------------
// Census population control.  When more than `cap` particles reach t_{n+1},
// every survivor is kept with probability p_q and reweighted by 1/p_q, where
// p_q = (cap - margin)/count rounded down to 11 significant bits
// (margin = ceil(4 sqrt(cap)) + 16, computed on the host).  The draw tests the
// survivor's own key mix64(thin_stream ^ hid) against p_q 2^64, so a
// survivor's fate does not depend on the others, and p_q sits on a coarse
// grid that a change of the count by a few particles does not move.  If more
// than cap survive the draw, the first cap in slot order are kept.
// ---------------------------------------------------------------------------
__global__ void k_thin_params(DevState* st, long long cap, long long margin) {
  if (threadIdx.x != 0 || st->halt) return;
  const unsigned long long cnt = st->alive;
  st->thin_overflow = 0;
  if (cnt <= (unsigned long long)cap) {
    st->thin_active = 0;
    st->thin_factor = 1.0;
    st->thin_mant = 0ull;
    st->thin_rshift = 64;
    return;
  }
  long long target = cap - margin;
  if (target < 1) target = 1;
  const double p = (double)target / (double)cnt;
  int k;
  const double m = frexp(p, &k);
  const double mant = floor(ldexp(m, 11));
  const double p_q = ldexp(mant, k - 11);
  st->thin_active = 1;
  st->thin_mant = (unsigned long long)mant;
  st->thin_rshift = 64 + (k - 11);
  st->thin_factor = 1.0 / p_q;
}

hipError_t launch_thin_params(DevState* st, long long cap, long long margin, hipStream_t s) {
  hipLaunchKernelGGL(k_thin_params, dim3(1), dim3(1), 0, s, st, cap, margin);
  return hipGetLastError();
}

long long census_tiles(long long n) { return (n + kKeepTile - 1) / kKeepTile; }

// One tile of kKeepTile candidates per block, read in rounds of 256 (slot
// base + r 256 + t in round r, thread t): each candidate's keep decision in
// place of its alive byte, the tile's kept count, and the cell of each kept
// candidate in a plain array (history id and cell share a 32-byte sector of
// the record, so the copy costs no extra read, and the ordering keys then
// read 4 bytes a slot instead of the records).
template <typename R>
__global__ __launch_bounds__(256) void k_census_keep(uint8_t* __restrict__ alive,
                                                     const StageRec<R>* __restrict__ stage,
                                                     long long n, uint64_t seed,
                                                     const DevState* st,
                                                     long long* __restrict__ tcount,
                                                     int32_t* __restrict__ cell) {
  if (st->halt) return;
  __shared__ int s_c[4];
  // the thinning keys' stream: (step, pass 2, population 2)
  const uint64_t thin_stream = stream_seed(seed, st->step, 2u, 2u, 0ull);
  const int act = st->thin_active;
  const unsigned long long mant = st->thin_mant;
  const int rs = st->thin_rshift;
  const long long base = (long long)blockIdx.x * kKeepTile;
  int cnt = 0;
  for (int r = 0; r < kKeepTile / 256; ++r) {
    const long long i = base + r * 256 + threadIdx.x;
    if (i >= n) break;
    int f = alive[i] ? 1 : 0;
    int c = 0;
    if (f) {
      c = stage[i].cell;
      if (act) {
        const unsigned long long key = mix64(thin_stream ^ stage[i].hid);
        const unsigned long long top = rs >= 64 ? 0ull : (key >> rs);
        f = top < mant ? 1 : 0;
        alive[i] = (uint8_t)f;
      }
    }
    cell[i] = f ? c : 0;
    cnt += f;
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if (__lane_id() == 0) s_c[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) tcount[blockIdx.x] = (long long)(s_c[0] + s_c[1] + s_c[2] + s_c[3]);
}

template <typename R>
hipError_t launch_census_keep(uint8_t* alive, const StageRec<R>* stage, long long n,
                              uint64_t seed, const DevState* st, long long* tcount,
                              int32_t* cell, hipStream_t s) {
  const long long tiles = census_tiles(n > 0 ? n : 1);
  hipLaunchKernelGGL(k_census_keep<R>, dim3((unsigned)tiles), dim3(256), 0, s, alive, stage, n,
                     seed, st, tcount, cell);
  return hipGetLastError();
}
template hipError_t launch_census_keep<double>(uint8_t*, const StageRec<double>*, long long,
                                               uint64_t, const DevState*, long long*, int32_t*,
                                               hipStream_t);
template hipError_t launch_census_keep<float>(uint8_t*, const StageRec<float>*, long long,
                                              uint64_t, const DevState*, long long*, int32_t*,
                                              hipStream_t);

// ---------------------------------------------------------------------------
// The census bank at t_{n+1}: the kept candidates (first cap in slot order)
// ordered by cell, a cell's candidates in slot order, so that the census
// particles of a cell form a contiguous cohort.  k_census_keys writes the
// kept candidates' (cell, slot) pairs in slot order; a stable LSD radix sort
// orders them by cell; k_census_gather copies the records (weights scaled by
// the thinning factor); k_cohort_ranks gives every particle its rank in its
// cell's cohort.  The count min(kept, cap) is read on the device.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long census_count(const long long* incl_last, long long cap) {
  const long long k = *incl_last;
  return k < cap ? k : cap;
}

// The tile's kept candidates, in slot order, at their places among all kept
// ones (the kept of earlier tiles first; rounds in order, the waves of a
// round in order, lanes in order), the first cap of them only; their cells
// come from the array the keep decisions left.
__global__ __launch_bounds__(256) void k_census_keys(const int32_t* __restrict__ cell,
                                                     const uint8_t* __restrict__ keep,
                                                     const long long* __restrict__ tcount,
                                                     const long long* __restrict__ tincl,
                                                     long long n, long long cap,
                                                     uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals,
                                                     const DevState* st) {
  if (st->halt) return;
  __shared__ int s_w[4];
  long long before = tincl[blockIdx.x] - tcount[blockIdx.x];  // kept in earlier tiles
  if (before >= cap || tcount[blockIdx.x] == 0) return;       // the same for the whole block
  const long long base = (long long)blockIdx.x * kKeepTile;
  const int w = threadIdx.x >> 6;
  for (int r = 0; r < kKeepTile / 256; ++r) {
    const long long i = base + r * 256 + threadIdx.x;
    const bool f = i < n && keep[i] != 0;
    const unsigned long long m = __ballot(f);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (__lane_id() == 0) s_w[w] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int v = 0; v < 4; ++v) {
      off += v < w ? s_w[v] : 0;
      tot += s_w[v];
    }
    const long long pos = before + off + below;
    if (f && pos < cap) {
      keys[pos] = (uint32_t)cell[i];
      vals[pos] = (uint32_t)i;
    }
    before += tot;
    __syncthreads();
  }
}

hipError_t launch_census_keys(const int32_t* cell, const uint8_t* keep, const long long* tcount,
                              const long long* tincl, long long n, long long cap, uint32_t* keys,
                              uint32_t* vals, const DevState* st, hipStream_t s) {
  const long long tiles = census_tiles(n > 0 ? n : 1);
  hipLaunchKernelGGL(k_census_keys, dim3((unsigned)tiles), dim3(256), 0, s, cell, keep, tcount,
                     tincl, n, cap, keys, vals, st);
  return hipGetLastError();
}

// Stable LSD radix sort of (key, value) pairs.  Keys below 2^b sort in
// P = ceil(b / 10) passes of ceil(b / P)-bit digits (1024^2 cells: two passes
// of 10 bits; 140^2: two of 8).  A tile of 256 rounds x 256 pairs per block,
// with as many rounds as give 16 pairs per digit value on average (16 rounds
// up to 8-bit digits, 64 for 10-bit), so that the scatter of a tile still
// writes runs of whole sectors; the pairs are read in rounds (pair base +
// r 256 + t in round r, thread t), in index order.
//   upsweep:   the tile's digit histogram -> hist[digit][tile]
//   scan:      inclusive scan of hist (digit-major): the pairs of digit d of
//              tile b start at incl[d][b] - hist[d][b]
//   downsweep: every pair's rank among the tile's earlier pairs of its digit
//              (rounds in order; in a round, the waves in order and the
//              lanes of a wave in order, lanes of one digit matched by
//              ballots), then the scatter to start + rank.
constexpr int kSortMaxBits = 10;
constexpr int kSortMaxDigits = 1 << kSortMaxBits;

static int sort_key_bits(long long n_keys_max) {
  int bits = 1;
  while (bits < 32 && (1ll << bits) < n_keys_max) ++bits;
  return bits;
}

int radix_passes(long long n_keys_max) {
  return (sort_key_bits(n_keys_max) + kSortMaxBits - 1) / kSortMaxBits;
}

static int sort_digit_bits(long long n_keys_max) {
  const int p = radix_passes(n_keys_max);
  return (sort_key_bits(n_keys_max) + p - 1) / p;
}

static int sort_rounds(int digit_bits) { return digit_bits <= 8 ? 16 : 16 << (digit_bits - 8); }

static long long sort_tiles(long long n, int digit_bits) {
  const long long tile = 256ll * sort_rounds(digit_bits);
  return (n + tile - 1) / tile;
}

long long radix_tiles(long long n) { return sort_tiles(n, 8); }

// Histogram entries for any digit width: digits x tiles is largest for the
// widest digits (1024 x ceil(cap / 16384) >= 256 x ceil(cap / 4096)).
size_t radix_hist_elems(long long cap) {
  size_t m = 0;
  for (int b = 8; b <= kSortMaxBits; ++b)
    m = std::max(m, ((size_t)1 << b) * (size_t)sort_tiles(cap > 0 ? cap : 1, b));
  return m;
}

__global__ __launch_bounds__(256) void k_radix_up(const uint32_t* __restrict__ keys,
                                                  const long long* incl_last, long long cap,
                                                  int shift, int bits, int rounds,
                                                  long long n_tiles,
                                                  long long* __restrict__ hist,
                                                  const DevState* st) {
  if (st->halt) return;
  __shared__ uint32_t h[kSortMaxDigits];
  const int n_dig = 1 << bits;
  const uint32_t mask = (uint32_t)n_dig - 1u;
  for (int d = threadIdx.x; d < n_dig; d += 256) h[d] = 0u;
  __syncthreads();
  const long long count = census_count(incl_last, cap);
  const long long base = (long long)blockIdx.x * 256 * rounds;
  for (int r = 0; r < rounds; ++r) {
    const long long i = base + r * 256 + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < n_dig; d += 256)
    hist[(long long)d * n_tiles + blockIdx.x] = (long long)h[d];
}

__global__ __launch_bounds__(256) void k_radix_down(const uint32_t* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout,
                                                    const long long* incl_last, long long cap,
                                                    int shift, int bits, int rounds,
                                                    long long n_tiles,
                                                    const long long* __restrict__ hist,
                                                    const long long* __restrict__ hincl,
                                                    const DevState* st) {
  if (st->halt) return;
  __shared__ long long s_start[kSortMaxDigits];  // first output index of each digit of this tile
  __shared__ uint32_t s_run[kSortMaxDigits];     // pairs of each digit in the earlier rounds
  __shared__ uint32_t s_wave[4][kSortMaxDigits]; // pairs of each digit in each wave of the round
  const int t = threadIdx.x, w = t >> 6;
  const int n_dig = 1 << bits;
  const uint32_t mask = (uint32_t)n_dig - 1u;
  for (int d = t; d < n_dig; d += 256) {
    const long long hb = (long long)d * n_tiles + blockIdx.x;
    s_start[d] = hincl[hb] - hist[hb];
    s_run[d] = 0u;
    for (int v = 0; v < 4; ++v) s_wave[v][d] = 0u;
  }
  __syncthreads();
  const long long count = census_count(incl_last, cap);
  const long long base = (long long)blockIdx.x * 256 * rounds;
  for (int r = 0; r < rounds; ++r) {
    const long long i = base + r * 256 + t;
    const bool ok = i < count;
    const uint32_t key = ok ? kin[i] : 0u;
    const uint32_t val = ok ? vin[i] : 0u;
    const int d = (int)((key >> shift) & mask);
    // lanes of this wave with the same digit (among the valid ones)
    unsigned long long peers = __ballot(ok);
    for (int b = 0; b < bits; ++b) {
      const unsigned long long m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(peers >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
    const bool lead = ok && below == 0u;  // the first lane of its digit in the wave
    const uint32_t n_peer = (uint32_t)__popcll(peers);
    if (lead) s_wave[w][d] = n_peer;
    __syncthreads();
    if (ok) {
      uint32_t before = s_run[d];
      for (int v = 0; v < w; ++v) before += s_wave[v][d];
      const long long o = s_start[d] + before + below;
      kout[o] = key;
      vout[o] = val;
    }
    __syncthreads();
    // each wave's leaders move their counts into the running totals (integer
    // adds: the order of the waves does not matter) and clear their entries
    if (lead) {
      atomicAdd(&s_run[d], n_peer);
      s_wave[w][d] = 0u;
    }
    __syncthreads();
  }
}

// Sorts the first min(*incl_last, cap) pairs of (k0, v0) by key (keys below
// key_bound); the result is in (k0, v0) after an even number of passes, in
// (k1, v1) after an odd number (radix_passes(key_bound)).
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                            const long long* incl_last, long long cap, long long key_bound,
                            long long* hist, long long* hincl, long long* scan_tmp,
                            const DevState* st, hipStream_t s) {
  const int passes = radix_passes(key_bound);
  const int bits = sort_digit_bits(key_bound);
  const int rounds = sort_rounds(bits);
  const long long tiles = sort_tiles(cap > 0 ? cap : 1, bits);
  for (int p = 0; p < passes; ++p) {
    uint32_t* ki = (p & 1) ? k1 : k0;
    uint32_t* vi = (p & 1) ? v1 : v0;
    uint32_t* ko = (p & 1) ? k0 : k1;
    uint32_t* vo = (p & 1) ? v0 : v1;
    hipLaunchKernelGGL(k_radix_up, dim3((unsigned)tiles), dim3(256), 0, s, (const uint32_t*)ki,
                       incl_last, cap, bits * p, bits, rounds, tiles, hist, st);
    hipError_t e = scan_inclusive_i64(hist, hincl, (1ll << bits) * tiles, scan_tmp, &st->halt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_down, dim3((unsigned)tiles), dim3(256), 0, s, (const uint32_t*)ki,
                       (const uint32_t*)vi, ko, vo, incl_last, cap, bits * p, bits, rounds, tiles,
                       (const long long*)hist, (const long long*)hincl, st);
  }
  return hipGetLastError();
}

// Blocks of the gather grid; each leaves the max |w| it wrote in bmax.
int census_compact_blocks(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < kCensusBlocks ? (b < 1 ? 1 : b) : kCensusBlocks);
}

template <typename R>
__global__ __launch_bounds__(256) void k_census_gather(const StageRec<R>* __restrict__ src,
                                                       const uint32_t* __restrict__ vals,
                                                       const long long* incl_last, long long cap,
                                                       StageRec<R>* __restrict__ dst,
                                                       const DevState* st,
                                                       double* __restrict__ bmax) {
  if (st->halt) return;
  __shared__ double s_mx[4];
  const R f = (R)st->thin_factor;
  const long long count = census_count(incl_last, cap);
  double mx = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (long long)gridDim.x * blockDim.x) {
    StageRec<R> rec = src[vals[k]];
    const R w = rec.w * f;
    rec.w = w;
    dst[k] = rec;
    mx = fmax(mx, fabs((double)w));
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if (__lane_id() == 0) s_mx[threadIdx.x >> 6] = mx;
  __syncthreads();
  // one plain store per block (a device-scope atomic per block on one
  // address serialises the blocks)
  if (threadIdx.x == 0) bmax[blockIdx.x] = fmax(fmax(s_mx[0], s_mx[1]), fmax(s_mx[2], s_mx[3]));
}

template <typename R>
hipError_t launch_census_gather(const StageRec<R>* src, const uint32_t* vals,
                                const long long* incl_last, long long cap, StageRec<R>* dst,
                                const DevState* st, double* bmax, hipStream_t s) {
  hipLaunchKernelGGL(k_census_gather<R>, dim3(census_compact_blocks(cap)), dim3(256), 0, s, src,
                     vals, incl_last, cap, dst, st, bmax);
  return hipGetLastError();
}
template hipError_t launch_census_gather<double>(const StageRec<double>*, const uint32_t*,
                                                 const long long*, long long, StageRec<double>*,
                                                 const DevState*, double*, hipStream_t);
template hipError_t launch_census_gather<float>(const StageRec<float>*, const uint32_t*,
                                                const long long*, long long, StageRec<float>*,
                                                const DevState*, double*, hipStream_t);

// Cohort ranks of a bank ordered by cell (cells[k] of its n = *count
// particles): start[c] = the first k of cell c, rank[k] = k - start[cells[k]].
__global__ void k_cohort_starts(const uint32_t* __restrict__ cells, const long long* count,
                                uint32_t* __restrict__ start, const DevState* st) {
  if (st->halt) return;
  const long long n = *count;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    if (k == 0 || cells[k] != cells[k - 1]) start[cells[k]] = (uint32_t)k;
}

__global__ void k_cohort_ranks(const uint32_t* __restrict__ cells, const long long* count,
                               const uint32_t* __restrict__ start, uint32_t* __restrict__ rank,
                               const DevState* st) {
  if (st->halt) return;
  const long long n = *count;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    rank[k] = (uint32_t)(k - (long long)start[cells[k]]);
}

hipError_t launch_cohort_ranks(const uint32_t* cells, const long long* count, long long n_max,
                               uint32_t* start, uint32_t* rank, const DevState* st,
                               hipStream_t s) {
  long long b = (n_max + 255) / 256;
  const int grid = (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
  hipLaunchKernelGGL(k_cohort_starts, dim3(grid), dim3(256), 0, s, cells, count, start, st);
  hipLaunchKernelGGL(k_cohort_ranks, dim3(grid), dim3(256), 0, s, cells, count,
                     (const uint32_t*)start, rank, st);
  return hipGetLastError();
}

// The cells of a bank's records (for the ranks of a loaded checkpoint).
template <typename R>
__global__ void k_bank_cells(const StageRec<R>* __restrict__ bank, long long n,
                             uint32_t* __restrict__ cells) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    cells[k] = (uint32_t)bank[k].cell;
}

template <typename R>
hipError_t launch_bank_cells(const StageRec<R>* bank, long long n, uint32_t* cells,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long b = (n + 255) / 256;
  const int grid = (int)(b < 4096 ? b : 4096);
  hipLaunchKernelGGL(k_bank_cells<R>, dim3(grid), dim3(256), 0, s, bank, n, cells);
  return hipGetLastError();
}
template hipError_t launch_bank_cells<double>(const StageRec<double>*, long long, uint32_t*,
                                              hipStream_t);
template hipError_t launch_bank_cells<float>(const StageRec<float>*, long long, uint32_t*,
                                             hipStream_t);

// Census count and max |w| of the new bank (max over the compaction blocks),
// and the end of the time step.
__global__ __launch_bounds__(256) void k_census_finish(DevState* st, const long long* tincl,
                                                       long long n_tiles, long long cap,
                                                       const double* bmax, int nb) {
  if (st->halt) return;
  __shared__ double s_mx[4];
  double mx = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) mx = fmax(mx, bmax[b]);
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if (__lane_id() == 0) s_mx[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const long long k = n_tiles > 0 ? tincl[n_tiles - 1] : 0;
  st->thin_overflow = k > cap ? 1 : 0;
  st->n_in = k > cap ? cap : k;
  st->n_kept = st->n_in;
  st->maxabs_w = fmax(fmax(s_mx[0], s_mx[1]), fmax(s_mx[2], s_mx[3]));
  st->step += 1;  // end of the time step: the step counter that seeds the point streams
}

hipError_t launch_census_finish(DevState* st, const long long* tincl, long long n_tiles,
                                long long cap, const double* bmax, hipStream_t s) {
  hipLaunchKernelGGL(k_census_finish, dim3(1), dim3(256), 0, s, st, tincl, n_tiles, cap, bmax,
                     census_compact_blocks(cap));
  return hipGetLastError();
}

}  // namespace slh
