// (Q)MC pass of the scatter-limited hybrid method (Sec. 2.3 of the paper):
// emission stratified by cell, tracking with at most n_lim scatters per
// history, or per-cell limits N_s(x) (implicit capture with sigma_a before
// the limit, attenuation with sigma_t after it), exact track-length tallies
// w (1 - e^{-sigma l}) / sigma per segment, and the census write of the remap
// pass.
//
// Execution model: a persistent grid sized to the device's occupancy.  Every
// lane owns one history at a time and, when it ends, takes the next work
// index of its wave's chunk of consecutive indices.  A wave whose chunk is
// used up takes the next one: on large passes (four or more chunks of
// kWorkChunk per wave) from the pass's counter, which balances the load; on
// smaller ones, where a shared counter would be contended, chunk w + k W of
// W waves, sized to about eight per wave.  (140^2 checkerboard, 2e6 items:
// passes 0.16 / 0.14 ms against 0.24 / 0.20 from the counter; 256^2 thick
// medium, 2e7 items: 1.27 ms from the counter against 1.41 cyclic.)  Lanes refill without waiting for
// the slowest history of their wave, and the histories of a wave start close
// together (the work index follows the cell order of the banks), so their
// material reads and tally adds meet in the caches.  The work index g maps to
// census particle g (g < n_in) or source particle g - n_in; every random
// number of a history is a pure function of its (stream, dimension, point
// index), so results do not depend on which lane or wave ran it.  Tallies and balance sums are fixed point with integer atomics
// and are therefore independent of the schedule.  Each lane adds into one of
// several private copies of the tally (summed afterwards), through a small
// cache of tally words per wave in LDS, so that simultaneous updates of a busy
// cell do not queue on one cache line.
#include <atomic>
#include "slh_common.hpp"
#include "sobol_dirs.inc"

namespace slh {

const uint32_t* sobol_table_host() { return slh_sobol_v; }

template <typename R> struct Real;
template <> struct Real<double> {
  using V2 = double2;
  static __device__ __forceinline__ void scpi(double x, double* s, double* c) {
    sincospi(x, s, c);
  }
  static __device__ __forceinline__ SrcRec<double>* src(const PassArgs& a) { return a.src64; }
  // w e^{-z} = w + w (e^{-z} - 1): the weight minus what the segment removed
  static __device__ __forceinline__ double attenuate(double w, double, double em) {
    return fma(w, em, w);
  }
  static __device__ __forceinline__ double2 mat(const PassArgs& a, int c) {
    return a.mat_id16 ? a.mtab64[a.mat_id16[c]] : a.mat64[c];
  }
  static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
  static __device__ __forceinline__ const StageRec<double>* in(const PassArgs& a) {
    return a.in64;
  }
  static __device__ __forceinline__ StageRec<double>* out(const PassArgs& a) { return a.out64; }
  static __device__ __forceinline__ void stage(StageRec<double>* p, double px, double py,
                                               double ox, double oy, double w, uint64_t hid,
                                               int cell) {
    double2* o = reinterpret_cast<double2*>(p);
    o[0] = make_double2(px, py);
    o[1] = make_double2(ox, oy);
    o[2] = make_double2(w, __longlong_as_double((long long)hid));
    o[3] = make_double2(__longlong_as_double((long long)(unsigned)cell), 0.0);
  }
  static __device__ __forceinline__ void put_src(SrcRec<double>* p, double px, double py,
                                                 double ox, double oy, double w, double trel,
                                                 double tau, int cell, uint32_t lidx) {
    double2* o = reinterpret_cast<double2*>(p);
    o[0] = make_double2(px, py);
    o[1] = make_double2(ox, oy);
    o[2] = make_double2(w, trel);
    o[3] = make_double2(tau, __longlong_as_double((long long)(((uint64_t)lidx << 32) |
                                                              (uint32_t)cell)));
  }
};
template <> struct Real<float> {
  using V2 = float2;
  static __device__ __forceinline__ void scpi(float x, float* s, float* c) {
    sincospif(x, s, c);
  }
  static __device__ __forceinline__ SrcRec<float>* src(const PassArgs& a) { return a.src32; }
  static __device__ __forceinline__ float attenuate(float w, float z, float) {
    return w * expf(-z);
  }
  static __device__ __forceinline__ float2 mat(const PassArgs& a, int c) {
    return a.mat_id16 ? a.mtab32[a.mat_id16[c]] : a.mat32[c];
  }
  static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
  static __device__ __forceinline__ const StageRec<float>* in(const PassArgs& a) {
    return a.in32;
  }
  static __device__ __forceinline__ StageRec<float>* out(const PassArgs& a) { return a.out32; }
  static __device__ __forceinline__ void stage(StageRec<float>* p, float px, float py, float ox,
                                               float oy, float w, uint64_t hid, int cell) {
    float4* o = reinterpret_cast<float4*>(p);
    o[0] = make_float4(px, py, ox, oy);
    o[1] = make_float4(w, __int_as_float(cell), __uint_as_float((unsigned)hid),
                       __uint_as_float((unsigned)(hid >> 32)));
  }
  static __device__ __forceinline__ void put_src(SrcRec<float>* p, float px, float py, float ox,
                                                 float oy, float w, float trel, float tau,
                                                 int cell, uint32_t lidx) {
    float4* o = reinterpret_cast<float4*>(p);
    o[0] = make_float4(px, py, ox, oy);
    o[1] = make_float4(w, trel, tau, __int_as_float(cell));
    o[2] = make_float4(__uint_as_float(lidx), 0.f, 0.f, 0.f);
    o[3] = make_float4(0.f, 0.f, 0.f, 0.f);  // the padding too: whole sectors
  }
};

enum { EV_CENSUS = 0, EV_COLLIDE = 1, EV_XFACE = 2, EV_YFACE = 3 };
enum { END_NONE = 0, END_CENSUS, END_LEAK, END_CUTOFF };

__device__ __forceinline__ double maxabs4(const double* q) {
  return fmax(fmax(fabs(q[0]), fabs(q[1])), fmax(fabs(q[2]), fabs(q[3])));
}

// Bilinear interpolation of nodal values (nodes (0,0),(1,0),(0,1),(1,1)) at
// local coordinates (a, b); equal corners give exactly q[0].
__device__ __forceinline__ double bilinear(const double* q, double a, double b) {
  return q[0] + a * (q[1] - q[0]) + b * (q[2] - q[0]) + a * b * (q[0] - q[1] - q[2] + q[3]);
}

// Cell of source particle s: descend the count tree (leaf i = n_i, exact
// integers) with target s + 1/2, going left while the target is below the
// left count, else subtracting it and going right.  Particles are numbered
// in cell order, so this finds the cell j with P_j <= s < P_j + n_j
// (P_j = counts of the cells before j), and l = s - P_j.  A thread descends
// NP particles' paths together, one level at a time, so that their loads of
// the lower levels (from global memory) are in flight at once.
constexpr int kTreeTop = 1024;  // nodes [0, kTreeTop) of the tree are staged in LDS

struct CellPick {
  long long cell;
  uint32_t l;
};

template <int NP>
__device__ __forceinline__ void count_pick_n(const double* __restrict__ t,
                                             const double* __restrict__ top, long long L,
                                             const long long* s, CellPick* out) {
  double target[NP];
  long long k[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    target[j] = (double)s[j] + 0.5;
    k[j] = 1;
  }
  // at the level of nodes [lev, 2 lev) the children [2 lev, 4 lev) are all
  // in LDS or all in global memory
  for (long long lev = 1; lev < L; lev <<= 1) {
    const bool in_lds = 4 * lev <= kTreeTop;
    double2 lr[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j)
      lr[j] = in_lds ? make_double2(top[2 * k[j]], top[2 * k[j] + 1])
                     : reinterpret_cast<const double2*>(t)[k[j]];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      if (target[j] < lr[j].x || lr[j].y == 0.0) {  // (an empty right subtree is never reached)
        k[j] = 2 * k[j];
      } else {
        target[j] -= lr[j].x;
        k[j] = 2 * k[j] + 1;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NP; ++j)
    out[j] = CellPick{k[j] - L, (uint32_t)target[j]};  // target = s - P_j + 1/2
}

// One fixed-point tally add.  XCD-local copies are only ever added to by
// workgroups of one XCD, so a workgroup-scope atomic, resolved in that XCD's
// L2, is exact; kernel boundaries write the L2 back before the copies are
// summed.  Otherwise a device-scope atomic.
__device__ __forceinline__ void tally_add(unsigned long long* p, unsigned long long v, int xl) {
  if (xl) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else atomicAdd(p, v);
}

// Work indices a wave takes from the pass's counter at a time (on the
// 1024x1024 solve 1024 gave the shortest passes: 64 queue on the counter,
// 16384 balance worse).
constexpr long long kWorkChunk = 1024;

// Tally-word cache of a wave in LDS: kTcSlots slots of (word address, pending
// sum).  A lane's add goes to the slot its word hashes to: into the slot's
// sum when the slot holds that word or is free (claimed with a compare and
// swap), else straight to the tally.  Every kTcFlush loop iterations, and at
// the end, the wave adds each held sum to its word and frees the slots.
// The histories of a wave start on neighbouring work items (cell order) and
// stay near each other, so many adds of a busy region meet in the cache
// instead of queueing at the same L2 lines; integer sums make the result the
// same as with one atomic per add.  512 slots per wave (32 KB per block) keep
// three blocks per compute unit.
constexpr int kTcSlots = 512;
constexpr int kTcFlush = 16;

__device__ __forceinline__ int tc_slot(unsigned long long ad) {
  // word index plus the 8 MB-aligned high bits, so that copies of one cell
  // (a power of two apart) fall in different slots
  return (int)(((ad >> 3) + (ad >> 23) * 37ull) & (unsigned long long)(kTcSlots - 1));
}

// Copies of a tracking block's balance in LDS (odd stride: the copies start
// in different banks).
constexpr int kBalCopies = 8;
constexpr int kBalStride = 2 * B_NFIELDS + 1;

// Adds v, in fixed point (hi, lo) of unit 1/inv_W, to balance field f.
__device__ __forceinline__ void bal_add(unsigned long long* bal, int f, double v, double inv_W) {
  long long hi, lo;
  fix_split(v, inv_W, hi, lo);
  atomicAdd(&bal[2 * f], (unsigned long long)hi);
  atomicAdd(&bal[2 * f + 1], (unsigned long long)lo);
}

// A value every lane of the wave holds alike (read from the solver state,
// which the compiler cannot take as uniform), moved to scalar registers so
// that it takes no vector register in the tracking loop.
__device__ __forceinline__ long long wave_uniform(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double wave_uniform(double v) {
  return __longlong_as_double(wave_uniform((long long)__double_as_longlong(v)));
}
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Emission of the pass's source particles (Sec. 2.3: birth proportional to
// q, isotropic direction, weights that integrate q in expectation),
// stratified by cell: cell j emits the n_j particles of the emission plan
// (floor(r_j) or floor(r_j) + 1, E[n_j] = r_j = M_j / w_q), numbered in cell
// order.  Particle l of cell j takes its points from the cell's stream at
// index l: position (dims 0-1), birth time (dim 2), direction (dims 3-4,
// sincospi), the first optical depth (dim 5) when the pass allows scatters,
// and weight w_q q(x,y) / qbar_j, qbar_j the cell's power-of-two majorant of
// |q| (so |w| <= w_q; the expected weight of the cell is r_j w_q mean(q) /
// qbar_j = A dt mean(q), or A mean(q) per unit time in steady state, where
// every particle starts at time 0).
//
// A thread emits runs of consecutive particles, up to kEmitRun of them when
// the plan has that many per thread of the grid (one otherwise, so that a
// small plan still spreads over the whole grid).  With tens of particles per
// cell a run nearly always lies in one emitter: the descents of its first
// and last particles then show it, and the emitter's stream and
// per-dimension scramble seeds are computed once for the run.  A run that
// spans emitters descends the tree for each of its inner particles.
constexpr long long kEmitRun = 8;

template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_emit(PassArgs a) {
  if (a.st->halt) return;
  __shared__ uint32_t s_sobol[kSobolNibbleWords];
  __shared__ double s_top[kTreeTop];
  sobol_nibbles_fill(a.sobol, s_sobol, threadIdx.x, blockDim.x);
  {
    const long long ntop = 2 * a.tree_L < kTreeTop ? 2 * a.tree_L : kTreeTop;
    for (int k = threadIdx.x; k < kTreeTop; k += blockDim.x)
      s_top[k] = (k >= 1 && k < ntop) ? a.ctree[k] : 0.0;
  }
  __syncthreads();
  const long long n_emit = a.st->n_emit;  // the plan's count, clamped to the bank
  const uint64_t step = a.st->step;
  const double wq = a.st->wq[KIND - 1];
  const R hx = (R)a.hx, hy = (R)a.hy, dt_birth = (R)a.dt_birth;
  SrcRec<R>* const b = Real<R>::src(a);
  const long long T = (long long)gridDim.x * blockDim.x;
  const long long run = n_emit / T < 1 ? 1 : (n_emit / T > kEmitRun ? kEmitRun : n_emit / T);
  for (long long r0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * run; r0 < n_emit;
       r0 += run * T) {
    const long long r1 = (r0 + run < n_emit ? r0 + run : n_emit) - 1;
    long long sj[2] = {r0, r1};
    CellPick pk[2];
    count_pick_n<2>(a.ctree, s_top, a.tree_L, sj, pk);
    const bool one = pk[0].cell == pk[1].cell;
    long long cur = -1;  // the emitter whose stream and seeds are held
    uint64_t stream = 0;
    uint32_t sd[6];
#pragma unroll 1
    for (long long s = r0; s <= r1; ++s) {
      CellPick pc;
      if (one) pc = CellPick{pk[0].cell, pk[0].l + (uint32_t)(s - r0)};
      else if (s == r0) pc = pk[0];
      else if (s == r1) pc = pk[1];
      else count_pick_n<1>(a.ctree, s_top, a.tree_L, &s, &pc);
      const long long ci = pc.cell;  // the emitter: a cell, or a boundary face after them
      const uint32_t l = pc.l;
      if (ci != cur) {
        cur = ci;
        stream = stream_seed(a.seed, step, (uint32_t)KIND, 0u, (uint64_t)ci);
#pragma unroll
        for (int d = 0; d < 6; ++d) sd[d] = point_seed(stream, (uint32_t)d);
      }
      const R u1 = PointU<R>::u(point_u32s(s_sobol, a.points, stream, sd[0], 0u, l));
      const R u2 = PointU<R>::u(point_u32s(s_sobol, a.points, stream, sd[1], 1u, l));
      const R u3 = PointU<R>::u(point_u32s(s_sobol, a.points, stream, sd[2], 2u, l));
      const R u4 = PointU<R>::u(point_u32s(s_sobol, a.points, stream, sd[3], 3u, l));
      const R tau = a.n_lim > 0
                        ? -log(PointU<R>::u(point_u32s(s_sobol, a.points, stream, sd[5], 5u, l)))
                        : (R)0;
      if (ci < a.n_cells) {
        const R u5 = PointU<R>::u(point_u32s(s_sobol, a.points, stream, sd[4], 4u, l));
        const R sn = (R)2 * sqrt(u4 * ((R)1 - u4));
        R sp, cp;
        Real<R>::scpi((R)2 * u5, &sp, &cp);
        const double* q = a.qn + 4 * ci;
        const double wscale = wq / pow2_ceil(maxabs4(q));  // exact: a power-of-two ratio
        const R w = (R)(bilinear(q, (double)u1, (double)u2) * wscale);
        Real<R>::put_src(b + s, hx * u1, hy * u2, sn * cp, sn * sp, w, u3 * dt_birth, tau,
                         (int)ci, l);
      } else {
        // entering through boundary face f (the inflow G): uniform along the
        // face (dim 0) and in time (dim 1), the cosine law about the inward
        // normal, mu = sqrt(u) (dim 2), the in-plane tangential component
        // sqrt(1 - mu^2) cos(2 pi u) (dim 3); weight w_q G_f / pow2_ceil(|G_f|)
        int k;
        const int f = (int)(ci - a.n_cells);
        const int side = face_side(f, a.nx, a.ny, &k);
        const R mu = sqrt(u3);
        R sp, cp;
        Real<R>::scpi((R)2 * u4, &sp, &cp);
        const R tg = sqrt((R)1 - u3) * cp;
        const double G = a.em.inflow[f];
        const R w = (R)(G * (wq / pow2_ceil(fabs(G))));
        R px, py, ox, oy;
        if (side < 2) {
          px = side == 0 ? (R)0 : hx;
          py = hy * u1;
          ox = side == 0 ? mu : -mu;
          oy = tg;
        } else {
          px = hx * u1;
          py = side == 2 ? (R)0 : hy;
          oy = side == 2 ? mu : -mu;
          ox = tg;
        }
        Real<R>::put_src(b + s, px, py, ox, oy, w, u2 * dt_birth, tau, (int)ci, l);
      }
    }
  }
}

template <typename R, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mc_pass(PassArgs a) {
  if (a.st->halt) return;
  // Block balance in kBalCopies LDS copies picked by lane: with a per-lane
  // address the adds are plain LDS atomics, where one shared address would
  // make the compiler serialise them over the active lanes in a scalar loop.
  // The emitted weight is not added per history: it is the sum of the source
  // and census-in weights (exact in fixed point).
  __shared__ unsigned long long s_bal[kBalCopies * kBalStride];
  __shared__ unsigned long long s_cnt[4];
  __shared__ uint32_t s_sobol[kSobolNibbleWords];
  __shared__ unsigned long long s_tc_tag[4 * kTcSlots];  // four waves per block
  __shared__ unsigned long long s_tc_sum[4 * kTcSlots];
  for (int k = threadIdx.x; k < 4 * kTcSlots; k += blockDim.x) {
    s_tc_tag[k] = 0ull;
    s_tc_sum[k] = 0ull;
  }
  for (int k = threadIdx.x; k < kBalCopies * kBalStride; k += blockDim.x) s_bal[k] = 0ull;
  if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0ull;
  sobol_nibbles_fill(a.sobol, s_sobol, threadIdx.x, blockDim.x);
  __syncthreads();

  DevState* st = a.st;
  const int lane = __lane_id();
  const long long n_in = wave_uniform(st->n_in);
  const long long n_emit = wave_uniform(st->n_emit);  // the plan's count, clamped to the bank
  const unsigned long long n_tot = (unsigned long long)(n_in + n_emit);
  const double w_q = wave_uniform(st->wq[KIND - 1]);
  const R w_cut = wave_uniform((R)(a.w_cut_rel * w_q));
  const double inv_T = wave_uniform(st->inv_T);
  const double inv_W = wave_uniform(st->inv_W);
  const uint64_t step = (uint64_t)wave_uniform((long long)st->step);
  const R hx = (R)a.hx, hy = (R)a.hy, dt = (R)a.dt, c = (R)a.c;
  const R INF = Real<R>::inf();
  const StageRec<R>* const bin = Real<R>::in(a);
  StageRec<R>* const bout = Real<R>::out(a);
  const int n_lim = a.n_lim;

  bool have = false;
  const long long gtid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long q_next = 0, q_end = 0;  // the wave's current chunk of work indices (uniform)
  bool q_done = false;              // no chunk is left for this wave
  const long long n_wv = (long long)gridDim.x * (blockDim.x / 64);
  const long long per_wave = (long long)n_tot / n_wv;
  const bool q_dyn = per_wave >= 4 * kWorkChunk;  // chunks from the pass's counter
  const long long chunk = q_dyn ? kWorkChunk : (per_wave / 8 > 16 ? per_wave / 8 : 16);
  // (the wave's index, read as a wave-uniform value so that the chunk state
  // stays in scalar registers)
  long long q_chunk = (long long)blockIdx.x * (blockDim.x / 64) +
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // tally copy of this lane: within the copies of the workgroup's XCD when
  // the copies are XCD-local (the hardware XCC id, not the dispatch order,
  // decides which L2 resolves the adds)
  const int xl = a.xcd_local;
  unsigned xcc = 0;
  if (xl) asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  const int per = xl ? a.n_copies / kNumXcd : a.n_copies;
  const long long my_copy =
      ((xl ? (long long)(xcc % kNumXcd) * per : 0ll) + gtid % per) * a.copy_stride;
  long long g = 0;
  unsigned long long* p_ptr = nullptr;  // the lane's pending tally word and sum
  unsigned long long p_val = 0ull;
  // material of the history's current cell, loaded when the history starts
  // and, after a face crossing, at the end of the iteration, so that the
  // gather is in flight while the loop turns around
  typename Real<R>::V2 m_cur;
  m_cur.x = (R)0;
  m_cur.y = (R)0;
  R px = 0, py = 0, ox = 0, oy = 0, w = 0, trel = 0, tau = 0;
  R iox = 0, ioy = 0;  // 1/ox, 1/oy (0 for a zero component)
  int ix = 0, iy = 0, n = 0;
  uint64_t stream = 0, hid = 0;
  uint32_t pidx = 0, dcur = 0, seg_p = 0;
  double w0 = 0.0, acc_abs = 0.0, acc_sca = 0.0;
  bool from_census = false;
  unsigned int lane_seg = 0, lane_hist = 0, lane_alive = 0, lane_killed = 0, lane_bad = 0;
  unsigned long long* my_bal = s_bal + (lane % kBalCopies) * kBalStride;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave in the block
  unsigned long long* const tc_tag = s_tc_tag + wv * kTcSlots;
  unsigned long long* const tc_sum = s_tc_sum + wv * kTcSlots;
  int tc_it = 0;
  // the wave's held sums to their words (all lanes of the wave together)
  auto tc_flush = [&]() __attribute__((always_inline)) {
    for (int k = lane; k < kTcSlots; k += 64) {
      const unsigned long long tg = tc_tag[k];
      if (tg) {
        tally_add((unsigned long long*)tg, tc_sum[k], xl);
        tc_tag[k] = 0ull;
        tc_sum[k] = 0ull;
      }
    }
  };

  for (;;) {
    // idle lanes take the next indices of the wave's chunk, in lane order; a
    // used-up chunk is replaced by the wave's next one
    bool fresh = false;
    if (__any(!have)) {
      if (q_next >= q_end && !q_done) {
        unsigned long long base = 0ull;
        if (q_dyn) {
          if (lane == 0) base = atomicAdd(&st->work, (unsigned long long)chunk);
          base = (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)base) |
                 ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                      (int)(unsigned)(base >> 32)) << 32);
        } else {
          base = (unsigned long long)(q_chunk * chunk);
          q_chunk += n_wv;
        }
        q_next = base < n_tot ? (long long)base : (long long)n_tot;
        q_end = base + chunk < n_tot ? (long long)(base + chunk) : (long long)n_tot;
        q_done = base + chunk >= n_tot;
      }
      const unsigned long long need = __ballot(!have);
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
      const long long avail = q_end - q_next;
      if (!have && (long long)rank < avail) {
        g = q_next + rank;
        fresh = true;
      }
      q_next += (long long)__popcll(need) < avail ? (long long)__popcll(need) : avail;
    }
    if (fresh) {
      have = true;
      lane_hist++;
      seg_p = 0;
      acc_abs = 0.0;
      acc_sca = 0.0;
      n = 0;
      if (g < n_in) {
        // census particle at the start of the step, counter reset
        from_census = true;
        const StageRec<R> rec = bin[g];
        px = rec.px; py = rec.py; ox = rec.ox; oy = rec.oy; w = rec.w;
        const int cell = rec.cell;
        ix = cell % a.nx; iy = cell / a.nx;
        hid = rec.hid;
        trel = (R)0;
        // census_qmc: its cell's census cohort, the cell's census stream at
        // the particle's rank in the cohort (the bank is ordered by cell);
        // else its own stream, keyed by its identity, at point index 0
        if (KIND == 1 && n_lim > 0) {
          stream = stream_seed(a.seed, step, (uint32_t)KIND, 1u,
                               a.census_qmc ? (uint64_t)cell : hid);
          pidx = a.census_qmc ? a.in_rank[g] : 0u;
        } else {
          stream = 0ull;
          pidx = 0u;
        }
        dcur = 0;
      } else {
        // source particle, emitted by k_emit
        from_census = false;
        const SrcRec<R> sr = Real<R>::src(a)[g - n_in];
        px = sr.px; py = sr.py; ox = sr.ox; oy = sr.oy; w = sr.w;
        trel = sr.trel;
        tau = sr.tau;
        const int cell = sr.cell;  // the emitter: a cell, or a boundary face after them
        pidx = sr.lidx;
        if (cell < a.n_cells) {
          ix = cell % a.nx; iy = cell / a.nx;
        } else {  // the cell inside boundary face f
          int k;
          const int side = face_side(cell - (int)a.n_cells, a.nx, a.ny, &k);
          ix = side < 2 ? (side == 0 ? 0 : a.nx - 1) : k;
          iy = side < 2 ? k : (side == 2 ? 0 : a.ny - 1);
        }
        // the emitter's stream at the particle's index in it
        stream = stream_seed(a.seed, step, (uint32_t)KIND, 0u, (uint64_t)cell);
        hid = history_id(step, cell, pidx);
        dcur = 6;  // dims 0-4 emission, 5 the first optical depth
      }
      iox = ox != (R)0 ? (R)1 / ox : (R)0;
      ioy = oy != (R)0 ? (R)1 / oy : (R)0;
      w0 = (double)w;
      m_cur = Real<R>::mat(a, iy * a.nx + ix);
      if (from_census && n_lim > 0) {
        tau = -log(PointU<R>::u(point_u32n(s_sobol, a.points, stream, 0u, pidx)));
        dcur = 1;
      }
    }
    if (!__any(have)) {
      if (p_ptr) tally_add(p_ptr, p_val, xl);  // the last pending add
      tc_flush();
      break;
    }
    // this iteration's tally word and value (none for an idle lane)
    unsigned long long* t_ptr = nullptr;
    unsigned long long t_val = 0ull;
    if (have) {

      // ---- one segment ----
      const int cell = iy * a.nx + ix;
      const R ss = m_cur.x, sa = m_cur.y, stt = sa + ss;
      const bool pre = n < (a.ns_cell ? a.ns_cell[cell] : n_lim);
      R d_cen = c * (dt - trel);
      if (d_cen < (R)0) d_cen = (R)0;
      R d_col = INF;
      if (pre && ss > (R)0) { d_col = tau / ss; if (d_col < (R)0) d_col = (R)0; }
      R d_x = INF, d_y = INF;
      if (ox > (R)0) d_x = (hx - px) * iox; else if (ox < (R)0) d_x = -px * iox;
      if (oy > (R)0) d_y = (hy - py) * ioy; else if (oy < (R)0) d_y = -py * ioy;
      if (d_x < (R)0) d_x = (R)0;
      if (d_y < (R)0) d_y = (R)0;
      R l = d_cen;
      int ev = EV_CENSUS;
      if (d_col < l) { l = d_col; ev = EV_COLLIDE; }
      if (d_x < l) { l = d_x; ev = EV_XFACE; }
      if (d_y < l) { l = d_y; ev = EV_YFACE; }

      const R sig = pre ? sa : stt;
      const R z = sig * l;
      const R em = expm1(-z);  // e^{-z} - 1
      const R contrib = (sig > (R)0) ? w * (-em) / sig : w * l;
      // the segment's tally word, added at the end of the iteration
      t_ptr = (pre ? a.Ta : a.Tb) + my_copy + kTallyStride * (long long)cell;
      {
        const double cd = (double)contrib;
        t_val = (unsigned long long)fix_round(cd, inv_T);
        acc_abs += (double)sa * cd;
        if (!pre) acc_sca += (double)ss * cd;
      }
      w = Real<R>::attenuate(w, z, em);
      if (pre && ss > (R)0) tau -= ss * l;
      trel += l / c;
      seg_p++;

      int end = END_NONE;
      if (ev == EV_CENSUS) {
        px += ox * l;
        py += oy * l;
        end = END_CENSUS;
      } else if (ev == EV_COLLIDE) {
        px += ox * l;
        py += oy * l;
        // isotropic re-emission, scatter counter n <- n + 1
        const R ua = PointU<R>::u(point_u32n(s_sobol, a.points, stream, dcur, pidx));
        const R ub = PointU<R>::u(point_u32n(s_sobol, a.points, stream, dcur + 1u, pidx));
        dcur += 2;
        const R sn = (R)2 * sqrt(ua * ((R)1 - ua));
        R sp, cp;
        Real<R>::scpi((R)2 * ub, &sp, &cp);
        ox = sn * cp;
        oy = sn * sp;
        iox = ox != (R)0 ? (R)1 / ox : (R)0;
        ioy = oy != (R)0 ? (R)1 / oy : (R)0;
        n++;
        if (n < n_lim) {
          tau = -log(PointU<R>::u(point_u32n(s_sobol, a.points, stream, dcur, pidx)));
          dcur++;
        }
      } else if (ev == EV_XFACE) {
        // a reflective side mirrors the direction; the history stays in its cell
        py += oy * l;
        if (ox > (R)0) {
          if (ix == a.nx - 1 && (a.bc & 2)) { px = hx; ox = -ox; iox = -iox; }
          else { ix++; px = (R)0; }
        } else {
          if (ix == 0 && (a.bc & 1)) { px = (R)0; ox = -ox; iox = -iox; }
          else { ix--; px = hx; }
        }
        if (ix < 0 || ix >= a.nx) end = END_LEAK;
      } else {
        px += ox * l;
        if (oy > (R)0) {
          if (iy == a.ny - 1 && (a.bc & 8)) { py = hy; oy = -oy; ioy = -ioy; }
          else { iy++; py = (R)0; }
        } else {
          if (iy == 0 && (a.bc & 4)) { py = (R)0; oy = -oy; ioy = -ioy; }
          else { iy--; py = hy; }
        }
        if (iy < 0 || iy >= a.ny) end = END_LEAK;
      }
      if (end == END_NONE && fabs(w) < w_cut) end = END_CUTOFF;
      if (end == END_NONE && seg_p >= a.max_segments) { end = END_CUTOFF; lane_killed++; }
      lane_seg++;
      // the next cell's material before the tally atomic: memory operations
      // complete in issue order, so the wait for the material at the next
      // segment does not include the atomic's round trip
      if (end == END_NONE && ev >= EV_XFACE) m_cur = Real<R>::mat(a, iy * a.nx + ix);

      if (end != END_NONE) {
        if (KIND == 2 && end == END_CENSUS && a.keep_census) {
          const long long slot = from_census ? g : a.out_src_base + (g - n_in);
          Real<R>::stage(bout + slot, px, py, ox, oy, w, hid, iy * a.nx + ix);
          a.alive[slot] = 1;
          lane_alive++;
        }
        // fold the history's balance into the block (fixed point, exact)
        const double wend = (double)w;
        if (!isfinite(wend) || !isfinite(acc_abs) || !isfinite(acc_sca)) lane_bad++;
        bal_add(my_bal, from_census ? B_CENSUS_IN_W : B_SOURCE_W, w0, inv_W);
        bal_add(my_bal, B_ABSORBED, acc_abs, inv_W);
        if (acc_sca != 0.0) bal_add(my_bal, B_SCATTERED, acc_sca, inv_W);
        bal_add(my_bal, end == END_CENSUS ? B_CENSUS : (end == END_LEAK ? B_LEAKED : B_CUTOFF),
                wend, inv_W);
        have = false;
      }
    }
    // A lane's consecutive adds to one word (segments that end in a
    // collision or at the census stay in their cell) are summed in registers;
    // the pending sum goes to the wave's cache when the lane moves to another
    // word.
    unsigned long long* f_ptr = nullptr;
    unsigned long long f_val = 0ull;
    if (t_ptr) {
      if (t_ptr == p_ptr) {
        p_val += t_val;
      } else {
        f_ptr = p_ptr;
        f_val = p_val;
        p_ptr = t_ptr;
        p_val = t_val;
      }
    }
    if (f_ptr) {
      const unsigned long long ad = (unsigned long long)f_ptr;
      const int slot = tc_slot(ad);
      unsigned long long tg = tc_tag[slot];
      if (tg == 0ull) {
        const unsigned long long old = atomicCAS(&tc_tag[slot], 0ull, ad);
        tg = old == 0ull ? ad : old;
      }
      if (tg == ad) atomicAdd(&tc_sum[slot], f_val);
      else tally_add(f_ptr, f_val, xl);
    }
    if (++tc_it == kTcFlush) {
      tc_it = 0;
      tc_flush();
    }
  }

  // wave totals of the integer counters, one atomic per wave
  unsigned long long v0 = lane_seg, v1 = lane_hist, v2 = lane_alive, v3 = lane_killed;
  for (int off = 32; off > 0; off >>= 1) {
    v0 += __shfl_xor(v0, off);
    v1 += __shfl_xor(v1, off);
    v2 += __shfl_xor(v2, off);
    v3 += __shfl_xor(v3, off);
  }
  if (lane_bad) atomicOr(&st->numeric, 2);
  if (lane == 0) {
    atomicAdd(&s_cnt[0], v0);
    atomicAdd(&s_cnt[1], v1);
    atomicAdd(&s_cnt[2], v2);
    atomicAdd(&s_cnt[3], v3);
  }
  __syncthreads();
  if (threadIdx.x < 2 * B_NFIELDS) {
    const int f = threadIdx.x >> 1, wd = threadIdx.x & 1;
    unsigned long long v = 0ull;
    for (int k = 0; k < kBalCopies; ++k) {
      const unsigned long long* b = s_bal + k * kBalStride;
      v += f == B_EMITTED ? b[2 * B_SOURCE_W + wd] + b[2 * B_CENSUS_IN_W + wd] : b[threadIdx.x];
    }
    if (v) atomicAdd(&st->bal[threadIdx.x], v);
  } else if (threadIdx.x >= 64 && threadIdx.x < 68) {
    const int k = threadIdx.x - 64;
    unsigned long long* dst = k == 0 ? &st->segments
                              : k == 1 ? &st->particles
                              : k == 2 ? &st->alive : &st->killed;
    if (s_cnt[k]) atomicAdd(dst, s_cnt[k]);
  }
}

// Blocks of the persistent tracking grid: as many as can be resident at once
// (occupancy x compute units), never more than the work needs.
int mc_pass_grid(bool fp32, int kind, long long max_work) {
  // solvers and servers are created from several threads: every thread that
  // finds the entry empty computes the same value and stores it atomically
  static std::atomic<int> cached[2][2];
  std::atomic<int>& slot = cached[fp32 ? 1 : 0][kind == 1 ? 0 : 1];
  int nb = slot.load(std::memory_order_relaxed);
  if (nb == 0) {
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e;
    if (kind == 1)
      e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_mc_pass<float, 1>, 256, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_mc_pass<double, 1>, 256, 0);
    else
      e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_mc_pass<float, 2>, 256, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_mc_pass<double, 2>, 256, 0);
    if (e != hipSuccess || per < 1) per = 2;
    if (cus < 1) cus = 256;
    nb = cus * per;
    slot.store(nb, std::memory_order_relaxed);
  }
  long long want = (max_work + 255) / 256;
  if (want > nb) want = nb;
  return (int)(want < 1 ? 1 : want);
}

hipError_t launch_emit(const PassArgs& a, bool fp32, hipStream_t s) {
  if (a.n_src <= 0) return hipSuccess;
  // at most 2048 blocks (each block first stages 24 KB of tables in LDS, six
  // blocks fit a compute unit); a thread takes its particles in runs
  long long b = (a.n_src + 255) / 256;
  const int grid = (int)(b < 2048 ? b : 2048);
  if (a.kind == 1) {
    if (fp32) hipLaunchKernelGGL((k_emit<float, 1>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_emit<double, 1>), dim3(grid), dim3(256), 0, s, a);
  } else {
    if (fp32) hipLaunchKernelGGL((k_emit<float, 2>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_emit<double, 2>), dim3(grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_mc_pass(const PassArgs& a, bool fp32, int grid, hipStream_t s) {
  if (a.kind == 1) {
    if (fp32) hipLaunchKernelGGL((k_mc_pass<float, 1>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_mc_pass<double, 1>), dim3(grid), dim3(256), 0, s, a);
  } else {
    if (fp32) hipLaunchKernelGGL((k_mc_pass<float, 2>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_mc_pass<double, 2>), dim3(grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// The tracking kernels' point function (nibble tables), one word per thread.
__global__ __launch_bounds__(256) void k_qmc_points(uint64_t stream, uint32_t dim0,
                                                    uint32_t nd, uint32_t idx0, uint32_t n,
                                                    int mode, const uint32_t* sobol,
                                                    uint32_t* out) {
  __shared__ uint32_t s_nib[kSobolNibbleWords];
  sobol_nibbles_fill(sobol, s_nib, threadIdx.x, blockDim.x);
  __syncthreads();
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * nd) return;
  const uint32_t k = (uint32_t)(t / nd), d = (uint32_t)(t % nd);
  out[t] = point_u32n(s_nib, mode, stream, dim0 + d, idx0 + k);
}

hipError_t launch_qmc_points(uint64_t stream, uint32_t dim0, uint32_t nd, uint32_t idx0,
                             uint32_t n, int mode, const uint32_t* sobol, uint32_t* out,
                             hipStream_t s) {
  const long long tot = (long long)n * nd;
  if (tot == 0) return hipSuccess;
  const int grid = (int)((tot + 255) / 256);
  hipLaunchKernelGGL(k_qmc_points, dim3(grid), dim3(256), 0, s, stream, dim0, nd, idx0, n,
                     mode, sobol, out);
  return hipGetLastError();
}

}  // namespace slh
