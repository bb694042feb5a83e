// Internal declarations of libslh: device-side helpers shared by the kernel
// translation units, the pass/step argument blocks and the launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slh {

// ---------------------------------------------------------------------------
// Point generator (Sec. 2.4 of the paper: low-discrepancy points used inside
// the existing inverse-CDF maps).  Sobol' words in natural index order,
// nested scrambling by the Laine-Karras hash permutation applied to the
// bit-reversed word (Burley 2020), streams and the pseudo-random mode from
// the SplitMix64 output function (Steele, Lea & Flood 2014).
// ---------------------------------------------------------------------------

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Stream of points for (time step, pass 1|2, population 0 source|1 census|2
// thinning, key): the key is the birth cell of a source particle and the
// history id of a census particle.
__host__ __device__ __forceinline__ uint64_t stream_seed(uint64_t seed, uint64_t step,
                                                          uint32_t pass, uint32_t pop,
                                                          uint64_t cohort) {
  uint64_t h = mix64(seed);
  h = mix64(h ^ step);
  h = mix64(h ^ (uint64_t)(pass * 16u + pop));
  return mix64(h ^ cohort);
}

__device__ __forceinline__ uint32_t nested_scramble(uint32_t x, uint32_t s) {
  x = __builtin_bitreverse32(x);
  x += s;
  x ^= x * 0x6c50b47cu;
  x ^= x * 0xb82f1e52u;
  x ^= x * 0xc7afe638u;
  x ^= x * 0x8d22f6e6u;
  return __builtin_bitreverse32(x);
}

constexpr int kSobolDims = 32;

// Point function of Sec. 2.4 (mode 0): the Sobol' word of (dim, index) is the
// XOR of the direction numbers V[dim][j] over the set bits j of the index,
// nested (Owen) scrambled with a per-(stream, dim) seed; mode 2 is the
// shifted Halton set below; dims beyond a set's table and the pseudo-random
// mode 1 hash (stream, dim, index).  The XOR runs over nibble
// tables: N[d][p][n] is the XOR of V[d][4p + k] over the set bits k of the
// 4-bit value n, so a word is the XOR of its index's eight nibble entries
// (eight lookups instead of a loop over the set bits).  N has kSobolDims x
// 8 x 16 words, built from V (kSobolDims x 32 words).
constexpr int kSobolNibbleWords = kSobolDims * 8 * 16;

__device__ __forceinline__ void sobol_nibbles_fill(const uint32_t* __restrict__ V, uint32_t* N,
                                                   int tid, int nthreads) {
  for (int e = tid; e < kSobolNibbleWords; e += nthreads) {
    const int d = e >> 7, pos = (e >> 4) & 7, n = e & 15;
    const uint32_t* v = V + d * 32 + 4 * pos;
    uint32_t x = 0;
    if (n & 1) x ^= v[0];
    if (n & 2) x ^= v[1];
    if (n & 4) x ^= v[2];
    if (n & 8) x ^= v[3];
    N[e] = x;
  }
}

__device__ __forceinline__ uint32_t sobol_word_nib(const uint32_t* N, uint32_t dim,
                                                   uint32_t index) {
  const uint32_t* t = N + dim * 128u;
  uint32_t x = 0;
#pragma unroll
  for (int pos = 0; pos < 8; ++pos) x ^= t[pos * 16 + ((index >> (4 * pos)) & 15u)];
  return x;
}

// Halton point set (the paper's generator, Sec. 2.4): coordinate d of point
// i is the radical inverse of i in the d-th prime base b, as the word
// floor(phi_b(i) 2^32).  With R the digit-reversed integer and D = b^K
// (K digits of i), phi_b(i) = R / D; the floor comes from two exact integer
// divisions, since R < D < 2^40.
constexpr int kHaltonDims = 32;
__device__ __forceinline__ uint32_t halton_u32(uint32_t dim, uint32_t index) {
  constexpr uint32_t kPrimes[kHaltonDims] = {2,  3,  5,  7,  11, 13, 17, 19, 23,  29,  31,
                                             37, 41, 43, 47, 53, 59, 61, 67, 71,  73,  79,
                                             83, 89, 97, 101, 103, 107, 109, 113, 127, 131};
  const uint32_t b = kPrimes[dim];
  uint64_t R = 0, D = 1;
  for (uint32_t i = index; i > 0; i /= b) {
    R = R * b + (uint64_t)(i % b);
    D *= b;
  }
  const uint64_t q1 = (R << 24) / D, r1 = (R << 24) % D;
  return (uint32_t)((q1 << 8) + ((r1 << 8) / D));
}

__device__ __forceinline__ uint32_t point_u32n(const uint32_t* N, int mode, uint64_t stream,
                                               uint32_t dim, uint32_t index) {
  if (mode == 0 && dim < (uint32_t)kSobolDims) {
    const uint32_t s = (uint32_t)(mix64(stream + dim) >> 32);
    return nested_scramble(sobol_word_nib(N, dim, index), s);
  }
  if (mode == 2 && dim < (uint32_t)kHaltonDims) {
    // randomised by a shift modulo 1 per (stream, dimension)
    const uint32_t s = (uint32_t)(mix64(stream + dim) >> 32);
    return halton_u32(dim, index) + s;
  }
  const uint64_t ctr = ((uint64_t)dim << 32) | (uint64_t)index;
  return (uint32_t)(mix64(stream ^ mix64(ctr)) >> 32);
}

// The same point with the scramble seed (Sobol') or shift (Halton) of
// (stream, dim) given, point_seed(stream, dim): every point of a stream and
// dimension shares it, so a caller that takes several points of one stream
// computes it once.
__device__ __forceinline__ uint32_t point_seed(uint64_t stream, uint32_t dim) {
  return (uint32_t)(mix64(stream + dim) >> 32);
}
__device__ __forceinline__ uint32_t point_u32s(const uint32_t* N, int mode, uint64_t stream,
                                               uint32_t seed, uint32_t dim, uint32_t index) {
  if (mode == 0 && dim < (uint32_t)kSobolDims)
    return nested_scramble(sobol_word_nib(N, dim, index), seed);
  if (mode == 2 && dim < (uint32_t)kHaltonDims) return halton_u32(dim, index) + seed;
  const uint64_t ctr = ((uint64_t)dim << 32) | (uint64_t)index;
  return (uint32_t)(mix64(stream ^ mix64(ctr)) >> 32);
}

// Smallest power of two >= v (v > 0), 0 for v = 0: the majorant of |q| in a
// cell is its largest corner value rounded up this way.
__host__ __device__ __forceinline__ double pow2_ceil(double v) {
  if (!(v > 0.0)) return 0.0;
  int e;
  const double m = frexp(v, &e);
  return (m == 0.5) ? v : ldexp(1.0, e);
}

// v rounded down to five significant bits (v > 0): the particle-weight
// quantum of the stratified emission, w_q = quantum(sum(M) / N_p).  Exact.
__host__ __device__ __forceinline__ double quantum5(double v) {
  if (!(v > 0.0)) return 0.0;
  int e;
  const double m = frexp(v, &e);
  return ldexp(floor(m * 32.0) / 32.0, e);
}

// Identity of source particle l of cell j born in time step `step`: a
// bijective mix of the packed (j, l), keyed by the step.
__host__ __device__ __forceinline__ uint64_t history_id(uint64_t step, long long j, uint32_t l) {
  return mix64((((uint64_t)j << 32) | (uint64_t)l) ^ mix64(step));
}

// Point 0 of a stream in dimension dim, without the Sobol' tables: the
// Sobol' word of index 0 is 0 and the Halton radical inverse of 0 is 0, so
// only the scramble or shift of (stream, dim) remains.  Equal to
// point_u32n(N, mode, stream, dim, 0) for every mode.
__device__ __forceinline__ uint32_t point_u32_first(int mode, uint64_t stream, uint32_t dim) {
  if ((mode == 0 && dim < (uint32_t)kSobolDims) || (mode == 2 && dim < (uint32_t)kHaltonDims)) {
    const uint32_t s = (uint32_t)(mix64(stream + dim) >> 32);
    return mode == 0 ? nested_scramble(0u, s) : s;
  }
  const uint64_t ctr = (uint64_t)dim << 32;
  return (uint32_t)(mix64(stream ^ mix64(ctr)) >> 32);
}

// u in (0,1) from a point word: FP64 keeps all 32 bits; FP32 keeps the top
// 23 bits so that (m + 1/2) 2^-23 is exact and never rounds to 0 or 1.
__device__ __forceinline__ double u01_f64(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }
__device__ __forceinline__ float u01_f32(uint32_t x) {
  return ((float)(x >> 9) + 0.5f) * 0x1p-23f;
}

template <typename R> struct PointU;
template <> struct PointU<double> {
  static __device__ __forceinline__ double u(uint32_t x) { return u01_f64(x); }
};
template <> struct PointU<float> {
  static __device__ __forceinline__ float u(uint32_t x) { return u01_f32(x); }
};

// ---------------------------------------------------------------------------
// Order-independent fixed-point accumulation.  Sums that must not depend on
// the schedule are kept as 64-bit integers in a power-of-two unit u chosen per
// pass from a bound B on every partial sum, u = 2^(ceil(log2 B) - 61), so no
// partial sum can overflow.  Integer addition is associative, so a sum is
// bitwise the same for any grid, schedule or order of its terms.
//   - Track-length tallies: one word per cell, each contribution rounded to
//     the nearest unit (error <= u/2 <= B 2^-62 per contribution).
//   - Balance sums (few, accumulated per block in LDS first): two words,
//     hi = trunc(v/u) and lo = rint(frac(v/u) 2^24), |lo| <= 2^24 per term.
// ---------------------------------------------------------------------------

constexpr double kLoScale = 16777216.0;  // 2^24

__device__ __forceinline__ long long fix_round(double v, double inv_unit) {
  return (long long)rint(v * inv_unit);
}

__device__ __forceinline__ void fix_split(double v, double inv_unit, long long& hi,
                                          long long& lo) {
  const double s = v * inv_unit;
  const double h = trunc(s);
  hi = (long long)h;
  lo = (long long)rint((s - h) * kLoScale);
}

__host__ __device__ __forceinline__ double fix_value(long long hi, long long lo, double unit) {
  const long long carry = lo >> 24;  // floor(lo / 2^24)
  hi += carry;
  lo -= carry << 24;
  return (double)hi * unit + (double)lo * (unit * (1.0 / kLoScale));
}

// Tally words are spaced kTallyStride apart.  One word per cell: on large
// meshes the tally copies' footprint in the L2 matters more than the
// sharing of cache lines between neighbouring cells' atomics.
constexpr int kTallyStride = 1;

// ---------------------------------------------------------------------------
// Layouts
// ---------------------------------------------------------------------------

// Census record of one particle: px, py, the position relative to the
// lower-left corner of its cell; ox, oy, the in-plane direction components;
// w, the weight; hid, the unique history id; cell.  64 B in FP64, 32 B in
// FP32, read and written as whole 16-byte words, so that a particle is one
// piece of one cache line.  The census bank is an array of these records,
// and the remap pass stages its census candidates in the same form (one
// record per slot) before the cap and compaction.  Layout (FP64): px py |
// ox oy | w hid | cell and padding; (FP32): px py ox oy | w cell hid.
template <typename R> struct StageRec;
template <> struct alignas(64) StageRec<double> {
  double px, py, ox, oy, w;
  uint64_t hid;
  int32_t cell, pad0;
  int64_t pad1;
};
template <> struct alignas(32) StageRec<float> {
  float px, py, ox, oy, w;
  int32_t cell;
  uint64_t hid;
};
static_assert(sizeof(StageRec<double>) == 64 && sizeof(StageRec<float>) == 32,
              "census record sizes");

// Source particle of one pass, written by the emission kernel and read once
// by the tracking kernel: position in the cell, direction, weight, birth time
// within the step, first optical depth (scatter-limited pass with N_s > 0
// only), cell and index within the cell (the particle's point index in its
// cell's stream).  One 64-byte record per particle in either precision, so
// that a history start reads one cache line rather than one line per field;
// the FP32 record is padded from 36 bytes to 64 so that the emission, whose
// threads each write a run of consecutive records, writes whole 64-byte
// sectors (48-byte records left partial sectors between a thread's
// consecutive records: 1.9x the record bytes in HBM writes).
template <typename R> struct SrcRec;
template <> struct alignas(64) SrcRec<double> {
  double px, py, ox, oy, w, trel, tau;
  int32_t cell;
  uint32_t lidx;
};
template <> struct alignas(64) SrcRec<float> {
  float px, py, ox, oy, w, trel, tau;
  int32_t cell;
  uint32_t lidx, pad0, pad1, pad2, pad3, pad4, pad5, pad6;
};
static_assert(sizeof(SrcRec<double>) == 64 && sizeof(SrcRec<float>) == 64,
              "source record sizes");

// Balance fields, each a two-word fixed-point sum.
enum BalField {
  B_EMITTED = 0, B_ABSORBED, B_SCATTERED, B_LEAKED, B_CENSUS, B_CUTOFF, B_SOURCE_W,
  B_CENSUS_IN_W, B_NFIELDS
};

// Device-resident state shared by the kernels of one solver.
// State of an iteration decided on the device.
struct IterState {
  int done;     // converged, iteration limit, or non-finite residual
  int conv;     // converged to the tolerance
  int iter;     // iterations done in this solve
  int bad;      // non-finite residual
  double dn2;   // |phi_new - phi_old|^2 of the last iteration (CG: |r|^2)
  double dn2_prev;  // the same of the iteration before (0 before the second)
  double nrm2;  // |phi_new|^2, or the whole-flux norm (CG: |b|^2)
  double rz;    // CG: r . z of the current iterate
  double beta;  // CG: beta of the next direction update
  double bb;    // CG: b . b
};

struct DevState {
  long long n_in;            // census-in bank size
  double maxabs_w;           // max |w| over the census-in bank
  unsigned long long alive;  // pass-2 census candidates
  long long n_kept;          // after the cap
  double thin_factor;        // count / cap or 1
  unsigned long long thin_mant;   // keep iff (key >> thin_rshift) < thin_mant
  int thin_rshift;
  int thin_active;
  int thin_overflow;              // more than cap survived the draw
  // set when a step's batch of source iterations ended before the iteration
  // did: every later kernel of that step and of the steps enqueued after it
  // returns at once, and the host runs them again (with a larger batch)
  int halt;
  // fixed-point units of the current pass (tally, balance) and inverses
  double unit_T, inv_T, unit_W, inv_W;
  unsigned long long work;      // work counter of the current pass
  unsigned long long segments;  // segments of the current pass
  unsigned long long particles; // histories of the current pass
  unsigned long long killed;    // histories stopped by the segment guard
  long long n_emit;             // source particles of the current pass
  // numeric faults of the current pass (bits): 1 a cell majorant or their
  // sum is not finite (no source particles are then emitted), 2 a history
  // ended with a non-finite weight or tally, 4 the plan exceeded the source
  // bank (clamped to it)
  int numeric;
  int pad2;
  unsigned long long bal[2 * B_NFIELDS];
  unsigned long long step;      // time step being computed (point streams, history ids)
  // source iteration of the collided solve (or the conjugate gradients of
  // the diffusion closing stage), kept on the device so that a batch of
  // iterations needs no host round trip: once si.done is set the remaining
  // iterations of the batch do nothing
  IterState si;
  // conjugate gradients of the diffusion correction inside each source
  // iteration (diffusion synthetic acceleration)
  IterState dsa;
  // emission plan of each pass kind (1, 2): the correctly rounded sum of the
  // cell majorants and the weight quantum
  double sumM[2];
  double wq[2];
  // diffusion corrections of the step whose conjugate gradients stopped at
  // the iteration limit before reaching their tolerance
  int dsa_unconv;
  int dsa_corrections;
  int dsa_iter_total;
  int dsa_iter_max;  // most conjugate-gradient iterations of one correction
  // totals since creation (or a checkpoint load), kept on the device so that
  // steps need no host round trip: segments of each pass kind, census-in
  // particles (each step's bank), census candidates written, histories
  // stopped by the segment guard, steps, steps whose census draw overflowed
  // the cap, steps whose source iteration stopped at its limit, and the OR of
  // every pass's numeric flags (DevState::numeric, plus 8: a non-finite
  // source-iteration residual, 16: the segment guard fired)
  unsigned long long acc_seg[2];
  unsigned long long acc_census_in, acc_census_out, acc_killed, acc_steps;
  unsigned long long acc_thin_overflow, acc_unconv;
  int acc_numeric;
  int pad3;
};

// Emitters of a pass beyond the cells: the boundary faces of a prescribed
// inflow G (n_faces = 2 (nx + ny) values, or none): the x_lo faces (index
// j), the x_hi faces, the y_lo faces (index i), the y_hi faces.  Face f's
// majorant is (side < 2 ? cx : cy) pow2_ceil(|G_f|), cx = (pi hy) tdt,
// cy = (pi hx) tdt with tdt the step (1 in steady state).
struct Emitters {
  const double* inflow;
  int nx, ny;
  long long n_faces;
  double cx, cy;
};

// Side of boundary face f (0 x_lo, 1 x_hi, 2 y_lo, 3 y_hi) and its index
// along the side.
__host__ __device__ __forceinline__ int face_side(int f, int nx, int ny, int* k) {
  if (f < ny) { *k = f; return 0; }
  if (f < 2 * ny) { *k = f - ny; return 1; }
  if (f < 2 * ny + nx) { *k = f - 2 * ny; return 2; }
  *k = f - 2 * ny - nx;
  return 3;
}

struct PassArgs {
  int nx, ny;
  // a history ends (census) at time dt after the start of the step, the
  // distance c (dt - t) ahead; source particles are born at u dt_birth
  // (dt_birth = dt; 0 in steady state, where dt is the path horizon, c = 1)
  double hx, hy, dt, c, dt_birth;
  int keep_census;       // remap pass: write the census-out particles
  const double2* mat64;  // (sigma_s, sigma_a) per cell
  const float2* mat32;
  // with few distinct materials: a 16-bit id per cell into (sigma_s,
  // sigma_a) tables, so that the gather of a segment touches 2 bytes per cell
  // of the mesh plus a small table; null otherwise
  const uint16_t* mat_id16;
  const double2* mtab64;
  const float2* mtab32;
  // emission, stratified by cell: cell i emits n_i = floor(r_i) or
  // floor(r_i) + 1 particles, r_i = M_i / w_q, w_q = quantum5(sum(M) / n_src)
  // (st->wq[kind - 1], with the exact sum st->sumM[kind - 1])
  const double* ctree;   // binary sum tree of the counts n_i (heap order; root: particles)
  long long tree_L;      // leaves start at tree_L (power of two >= the emitters)
  const double* qn;      // nodal source [cell][4]
  Emitters em;           // boundary faces of an inflow, emitters after the cells
  long long n_cells;
  long long n_src;       // N_p, the requested particles per pass
  long long src_cap;     // capacity of the source bank (the plan is clamped to it)
  double adt;            // cell area times dt (times 1 in steady state)
  uint64_t seed;         // the time step is read from st->step
  int kind;              // 1: scatter-limited leg, 2: scatter-free remap
  int n_lim;             // scatter limit of the pass (0 for kind 2); with
                         // per-cell limits, the largest of them
  const int* ns_cell;    // per-cell limits (unlimited as INT_MAX), or null
  int bc;                // reflective sides: 1 x_lo, 2 x_hi, 4 y_lo, 8 y_hi
  int points;            // 0 Sobol'-Owen, 1 pseudo-random
  const uint32_t* sobol; // direction numbers
  double w_cut_rel;
  unsigned int max_segments;
  // census: input bank and output slots (census index, or out_src_base +
  // source index), and the source particles, in the precision of the pass
  const StageRec<double>* in64;
  const StageRec<float>* in32;
  const uint32_t* in_rank;  // rank of each census particle in its cell's cohort
  int census_qmc;           // census histories: 1 cell cohorts, 0 a stream per history
  StageRec<double>* out64;
  StageRec<float>* out32;
  SrcRec<double>* src64;
  SrcRec<float>* src32;
  uint8_t* alive;
  long long out_src_base;  // slot of source particle s is out_src_base + s
  // tallies: n_copies private copies of one fixed-point word per cell (word
  // stride kTallyStride), copy c at offset c * copy_stride.  xcd_local: the
  // copies are split evenly over the eight XCDs, a workgroup adds only into
  // its own XCD's copies, and the adds are workgroup-scope atomics, which
  // the XCD's L2 resolves (device-scope atomics go past the L2)
  unsigned long long* Ta;
  unsigned long long* Tb;
  int n_copies;
  int xcd_local;
  long long copy_stride;
  DevState* st;
};

constexpr int kNumXcd = 8;  // XCDs of the device (hardware XCC ids 0..7)

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files)
// ---------------------------------------------------------------------------

hipError_t launch_emit(const PassArgs& a, bool fp32, hipStream_t s);
int mc_pass_grid(bool fp32, int kind, long long max_work);
hipError_t launch_mc_pass(const PassArgs& a, bool fp32, int grid, hipStream_t s);
hipError_t launch_qmc_points(uint64_t stream, uint32_t dim0, uint32_t nd, uint32_t idx0,
                             uint32_t n, int mode, const uint32_t* sobol, uint32_t* out,
                             hipStream_t s);
const uint32_t* sobol_table_host();

// Start of run d of a sweep layout (see DgArgs): the number of cells of an
// nx x ny mesh on the runs before it, sum over t < d of
// min(t, nx - 1) - max(0, t - (ny - 1)) + 1, in closed form.
__host__ __device__ __forceinline__ long long lay_run(int nx, int ny, int d) {
  const long long D = d, X = nx, Y = ny;
  const long long a = D <= X ? D * (D + 1) / 2 : X * (X + 1) / 2 + (D - X) * X;
  const long long b = D <= Y ? 0 : (D - Y) * (D - Y + 1) / 2;
  return a - b;
}

// Position of cell (i, j) in sweep layout A (anti = true) or B.
__host__ __device__ __forceinline__ long long lay_pos(int nx, int ny, int i, int j, bool anti) {
  const int d = anti ? i + j : i - j + ny - 1;
  const int lo = d - (ny - 1) > 0 ? d - (ny - 1) : 0;
  return lay_run(nx, ny, d) + (i - lo);
}

struct DgArgs {
  int nx, ny;
  double hx, hy;
  int n_dir;
  const double* dir;     // [m][3]: ox, oy, w
  // Sweep layouts: the cells of a direction whose components have the same
  // sign are visited along anti-diagonals (i + j constant), the others along
  // diagonals (i - j constant).  Layout A stores the cells anti-diagonal by
  // anti-diagonal (index d = i + j), layout B diagonal by diagonal (index
  // d = i - j + ny - 1); within either, cell i - lo(d) of the run, lo(d) =
  // max(0, d - (ny - 1)), and the run starts at lay_run(nx, ny, d).  A chunk
  // of a sweep is then a contiguous piece of its layout, so the sweep's loads
  // and its plane stores are whole cache lines.
  const int* fam_dirs;   // the directions of layout A in order, then those of B
  int fam_n;             // how many belong to layout A
  const double* sig_e;   // per cell, layout A then layout B (2 nx ny)
  const double* sig_s;   // per cell (row-major)
  const double* phi_post;// per cell
  const double* phi_pre; // per cell, or null: the stopping test's norm is then
                         // over phi_c alone, else over phi_c + phi_pre + phi_post
  double* phi_c;         // nodal [cell][4] (row-major): the collided iterate, updated in place
  double* src;           // nodal sigma_s/(4 pi)(phi_c + phi_post), layout A then B (8 nx ny)
  double* psi;           // [m][position][4] in the layout of direction m (psi_m;
                         // the reduction applies w_m)
  double* phi_fam;       // nodal sums of w_m psi_m over each layout's directions,
                         // layout A then B (8 nx ny)
  double* dnode;         // nodal phi^{k+1/2} - phi^k (row-major) for the diffusion
                         // correction (diffusion synthetic acceleration), or null
  const double* dirmat;  // [m][32]: A0 then F (uniform mesh)
  // table mode: material of each cell (layout A then B) and
  // [m][material][32] = B then G
  const int* mat_id;
  int n_mat;
  const double* coef;
  int cw;                // cells per chunk (a multiple of 64 cells_per_lane, at
                         // most 256 cells_per_lane)
  int n_chunks;          // dg_chunks(nx, ny, cw)
  int cells_per_lane;    // cells per sweeping and per loader lane: 1, 2 or 4
  // reflective sides (1 x_lo, 2 x_hi, 4 y_lo, 8 y_hi): the inflow of a
  // direction on such a side is the outflow of its mirror image (refl_x,
  // refl_y) from the previous iteration.  bnd holds two buffers of [n_dir]
  // [2 ny x traces | 2 nx y traces], written in iterations of the parity of
  // their index (null when no side reflects)
  int bc;
  const int* refl_x;
  const int* refl_y;
  double* bnd;
  DevState* st;          // si.done: skip the iteration; the reduction's decision
};
hipError_t launch_dg_tables(int n_dir, int n_mat, const double* dir, const double* sig_e_mat,
                            double hx, double hy, double* dirmat, double* coef, hipStream_t s);
long long dg_chunks(int nx, int ny, int cw);
size_t dg_sweep_lds_bytes(bool table, int cw, int n_mat, int nx, int ny);
// Start of a step's source iteration: phi_c = 0, iteration state reset, the
// first iterate's nodal source, reflected traces of the first sweep zeroed.
hipError_t launch_si_start(const DgArgs& a, int si_max, hipStream_t s);
// After a batch of source iterations: if the iteration has not stopped, the
// step halts (DevState::halt, and si.done so that no later iteration runs).
hipError_t launch_si_check(DevState* st, hipStream_t s);
// After a diffusion correction whose conjugate gradients were launched for
// fewer steps than their limit: a correction the steps left unfinished halts
// the step (it runs again with the full limit), as a short batch of source
// iterations does.
hipError_t launch_dsa_check(DevState* st, hipStream_t s);
// Diffusion synthetic acceleration: after the correction delta (per cell) is
// solved, phi += delta at every node, the next iterate's source, and the
// residual of phi^{k+1} - phi^k = dnode + delta, decided as after a plain
// reduction.
hipError_t launch_dsa_apply(const DgArgs& a, const double* delta, double* partials, int n_part,
                            double si_tol, int si_max, hipStream_t s);

// Diffusion closing stage (cell-centred finite volumes, Jacobi-preconditioned
// conjugate gradients).  Vectors are per cell; P holds two n-vectors (the
// search direction of the current and of the previous iteration, by parity);
// part_a / part_b hold 2 n_part block partials each.
struct CgArgs {
  int nx, ny;
  const double* diag;   // diagonal of the system (per unit cell area)
  const double* cE;     // coupling to the x+1 neighbour (0 across the boundary)
  const double* cN;     // coupling to the y+1 neighbour
  double *x, *r, *z, *P, *q;
  double *part_a, *part_b;
  int n_part;           // cg_partials(nx * ny)
  IterState* cs;        // the solve's state: st->si for the closing stage,
                        // st->dsa for the correction of a source iteration
  const int* gate;      // if not null and set (the source iteration is done),
                        // every kernel returns at once
};
int cg_partials(long long n);
hipError_t launch_diff_coef(int nx, int ny, const double2* mat, double tt, double hx, double hy,
                            int bc, double* diag, double* cE, double* cN, hipStream_t s);
// b = sigma_s phi_post, x = 0, and the state of a new solve (done at once when
// b = 0 or max_iter = 0); nothing while *halt is set
hipError_t launch_cg_start(const CgArgs& a, const double* sig_s, const double* phi_post,
                           int max_iter, const int* halt, hipStream_t s);
// the same for the diffusion correction of a source iteration: b = sigma_s
// times the cell average of dnode (phi^{k+1/2} - phi^k, four nodes per cell)
hipError_t launch_dsa_start(const CgArgs& a, const double* sig_s, const double* dnode,
                            int max_iter, hipStream_t s);
// the whole (remaining) solve in one workgroup, whatever the mesh size
hipError_t launch_cg_solve_one_block(const CgArgs& a, double tol, int max_iter, hipStream_t s);
// one iteration (nothing once the state says done); stops at |r| <= tol |b|.
// On meshes where cg_one_block holds, one call runs the whole solve.
bool cg_one_block(long long n);
hipError_t launch_cg_iteration(const CgArgs& a, double tol, int si_max, hipStream_t s);
hipError_t launch_cg_to_nodal(const CgArgs& a, double* phi_c, const int* halt, hipStream_t s);
hipError_t launch_dg_sweep(const DgArgs& a, bool table, hipStream_t s);
// One reduction of a source iteration: the direction sum of the planes (each
// layout's directions in order, then the two sums added) replaces phi_c in
// place, the next iterate's source is formed, and the residual decides
// st->si.done (n_part blocks, dg_reduce_partials).
hipError_t launch_dg_reduce(const DgArgs& a, double* partials, int n_part, double si_tol,
                            int si_max, hipStream_t s);
int dg_reduce_partials(long long n_nodes);

// util.hip
hipError_t launch_fill_u64(unsigned long long* p, long long n, unsigned long long v,
                           hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, long long n, uint8_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, long long n, double v, hipStream_t s);
// Pass set-up (counters, balance, fixed-point units from the bound on the
// emitted weight: particles (count-tree root) times w_q plus the census
// bound) with the clears of up to two tally arrays and a byte array.
hipError_t launch_pass_prep(DevState* st, const double* ctree, int kind, long long src_cap,
                            double cdt, unsigned long long* a, long long na,
                            unsigned long long* b, long long nb, uint8_t* c, long long nc,
                            hipStream_t s);
// phi = tally * unit / (A dt) for T0 -> phi0 and, when T1 is not null, T1 -> phi1.
hipError_t launch_tally_to_flux(const unsigned long long* T0, double* phi0,
                                const unsigned long long* T1, double* phi1, long long n,
                                int n_copies, long long copy_stride, const DevState* st,
                                double inv_adt, hipStream_t s);
hipError_t launch_remap_source(long long n, const double* q, const double* sig_s,
                               const double* phi_pre, const double* phi_post,
                               const double* phi_c, double* qn, const int* halt,
                               hipStream_t s);
long long tree_leaves(long long n_cells);
// Emission plan of a pass (the counts of the stratified emission): histogram
// of the cell majorants M_i = adt pow2_ceil(max corner |q_i|) by exponent,
// their exact sum rounded once to FP64 (st->sumM[kind - 1]), the weight
// quantum w_q (st->wq[kind - 1]), the counts
// n_i = floor(M_i / w_q) + [u_i < frac(M_i / w_q)] with u_i point 0 of the
// cell's count stream, and the count tree over them (root: particles).
// hist: kMajBins words, zero on entry and left zero (the last bin counts
// cells whose majorant is not finite).
constexpr int kMajBins = 2112;
hipError_t launch_emission_plan(const double* qn, long long n_cells, const Emitters& em,
                                double adt, long long n_src, uint64_t seed, int points, int kind,
                                unsigned long long* hist, double* ctree, DevState* st,
                                hipStream_t s);
// hist: kMajHistWords words (cells, x faces, y faces)
constexpr int kMajGroups = 3;
size_t scan_tmp_elems(long long n);
hipError_t scan_inclusive_i64(const long long* in, long long* out, long long n,
                              long long* tmp, const int* halt, hipStream_t s);
hipError_t launch_thin_params(DevState* st, long long cap, long long margin, hipStream_t s);
// Census candidates are processed in tiles of kKeepTile slots.
// launch_census_keep: each candidate's keep decision (alive and, with the cap
// active, its key test), stored in place of its alive byte, and the kept
// count of each tile (tcount, census_tiles(n) entries).
constexpr int kKeepTile = 4096;
long long census_tiles(long long n);
// It also copies each kept candidate's cell into cell (n entries; 0 for the
// others), read by the ordering keys in place of the records.
template <typename R>
hipError_t launch_census_keep(uint8_t* alive, const StageRec<R>* stage, long long n,
                              uint64_t seed, const DevState* st, long long* tcount,
                              int32_t* cell, hipStream_t s);
// The census bank at t_{n+1} (kept candidates, first cap in slot order,
// ordered by cell and within a cell by slot): (cell, slot) pairs of the kept
// candidates in slot order, then radix_sort_pairs by cell, then the gather of
// the records (weights times the thinning factor).  tincl: the inclusive
// scan of the tile counts, whose last entry (the kept total) bounds the count
// with cap.
hipError_t launch_census_keys(const int32_t* cell, const uint8_t* keep, const long long* tcount,
                              const long long* tincl, long long n, long long cap, uint32_t* keys,
                              uint32_t* vals, const DevState* st, hipStream_t s);
long long radix_tiles(long long n);
int radix_passes(long long n_keys_max);
size_t radix_hist_elems(long long cap);
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                            const long long* incl_last, long long cap, long long key_bound,
                            long long* hist, long long* hincl, long long* scan_tmp,
                            const DevState* st, hipStream_t s);
template <typename R>
hipError_t launch_census_gather(const StageRec<R>* src, const uint32_t* vals,
                                const long long* incl_last, long long cap, StageRec<R>* dst,
                                const DevState* st, double* bmax, hipStream_t s);
// bmax: kCensusBlocks doubles, the gather's per-block max |w|
// tincl: n_tiles inclusive tile counts (the last is the kept total)
hipError_t launch_census_finish(DevState* st, const long long* tincl, long long n_tiles,
                                long long cap, const double* bmax, hipStream_t s);
constexpr int kCensusBlocks = 2048;  // blocks of the gather grid at most
int census_compact_blocks(long long n);
// Ranks of the census particles in their cells' cohorts, for a bank ordered
// by cell (cells[k], k < *count); start: one entry per cell.
hipError_t launch_cohort_ranks(const uint32_t* cells, const long long* count, long long n_max,
                               uint32_t* start, uint32_t* rank, const DevState* st,
                               hipStream_t s);
template <typename R>
hipError_t launch_bank_cells(const StageRec<R>* bank, long long n, uint32_t* cells,
                             hipStream_t s);

}  // namespace slh
