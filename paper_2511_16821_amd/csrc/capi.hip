// Host side of libslh: argument validation, device memory, the S_N
// quadrature, the time-step driver (steps 1-4 of Sec. 2.2 of the paper) and
// the C ABI declared in include/slh.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <cstddef>
#include <new>
#include <string>
#include <vector>

#include "../../include/slh.h"
#include "slh_common.hpp"

using namespace slh;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static slh_status fail(slh_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

extern "C" const char* slh_last_error(void) { return g_err.c_str(); }

namespace slh {
// Sets the calling thread's message (the server hands a worker's message to
// the thread that collects the result).
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace slh

// Copies on the solver's stream and waits for it: no operation of the
// library uses the legacy default stream, which would have to wait for
// graph captures running on other threads' solvers.
#define COPY_SYNC(dst, src, n, kind)                                  \
  do {                                                                \
    HIP_TRY(hipMemcpyAsync(dst, src, n, kind, s->stream));            \
    HIP_TRY(hipStreamSynchronize(s->stream));                         \
  } while (0)

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(SLH_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(_e));     \
  } while (0)

// ---------------------------------------------------------------------------
// S_N product quadrature: N/2 positive Gauss-Legendre nodes of order N for
// Omega_z (weights doubled: -Omega_z has the same in-plane components) times
// 2N azimuths (m + 1/2) pi / N; N^2 directions, weights summing to 4 pi.
// Nodes by Newton's method on the Legendre three-term recurrence.
// ---------------------------------------------------------------------------
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static std::vector<double> product_quadrature(int order) {
  std::vector<double> x, w;
  gauss_legendre(order, x, w);
  std::vector<double> dirs;
  const int naz = 2 * order;
  for (int k = 0; k < order; ++k) {
    if (!(x[k] > 0.0)) continue;
    const double s = sqrt(1.0 - x[k] * x[k]);
    for (int m = 0; m < naz; ++m) {
      const double ph = (m + 0.5) * M_PI / order;
      dirs.push_back(s * cos(ph));
      dirs.push_back(s * sin(ph));
      dirs.push_back(2.0 * w[k] * M_PI / order);
    }
  }
  // group the directions by quadrant (stable), so that runs of equal-quadrant
  // directions can share a sweep workgroup
  const int n = (int)dirs.size() / 3;
  std::vector<double> out;
  out.reserve(dirs.size());
  for (int q = 0; q < 4; ++q)
    for (int m = 0; m < n; ++m) {
      const int qm = (dirs[3 * m] > 0.0 ? 0 : 1) + (dirs[3 * m + 1] > 0.0 ? 0 : 2);
      if (qm == q) out.insert(out.end(), dirs.begin() + 3 * m, dirs.begin() + 3 * m + 3);
    }
  return out;
}

// ---------------------------------------------------------------------------
// validation and sizes
// ---------------------------------------------------------------------------
struct Sizes {
  long long n_cells, n_p, cap, n_cand;
  long long n_faces;    // boundary faces emitting an inflow (0 without one)
  long long n_src_cap;  // source bank: at most n_p (1 + 1/16) + n_cells particles per pass
  int n_dir;
  int n_copies;  // private tally copies
  bool fp32;
  // DG sweep: table mode (per-(direction, material) coefficients staged in
  // LDS, n_mat distinct sigma_e) or cell mode; dg_cw cells per chunk, dg_q
  // of them per lane, dg_chunks chunks per sweep.
  int n_mat;
  bool dg_table;
  int dg_cw, dg_q;
  long long dg_chunks;
  bool diffusion;  // diffusion closing stage: no direction planes, CG vectors instead
  bool dsa;        // S_N with the diffusion correction: planes, CG vectors and dnode
  // tracking materials: with at most kMaxMatIds distinct (sigma_s, sigma_a)
  // pairs, a 16-bit id per cell and a table (n_mc_mat entries); else none
  // (n_mc_mat = 0) and the kernels read the per-cell arrays
  int n_mc_mat;
  size_t bytes;
};

constexpr int kMaxMatIds = 65535;

// Sorted distinct (sigma_s, sigma_a) pairs of the problem's cells.
static std::vector<std::pair<double, double>> material_pairs(const slh_problem* p) {
  const long long n = (long long)p->nx * p->ny;
  std::vector<std::pair<double, double>> v(n);
  for (long long i = 0; i < n; ++i) v[i] = std::make_pair(p->sigma_s[i], p->sigma_a[i]);
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

// tau/(c dt), the time closure of the collided solve; none in steady state
static double time_term(const slh_problem* p) {
  if (p->steady) return 0.0;
  const double tau = p->time_closure > 0.0 ? p->time_closure : 2.0;
  return tau / (p->c * p->dt);
}

static double sigma_e_of(const slh_problem* p, long long i) {
  return p->sigma_a[i] + p->sigma_s[i] + time_term(p);
}

// Steady state: the path length at which a history ends.  By default
// ln(1/w_cut_rel) / min sigma_a: a weight decays at least at rate min sigma_a
// (sigma_a before the limit, sigma_t after it) from at most w_q, so every
// history is below the cutoff w_cut_rel w_q by then.
static double horizon_of(const slh_problem* p) {
  if (p->horizon > 0.0) return p->horizon;
  const long long n = (long long)p->nx * p->ny;
  double mn = INFINITY;
  for (long long i = 0; i < n; ++i) mn = std::min(mn, p->sigma_a[i]);
  return log(1.0 / p->w_cut_rel) / mn;
}

// Sorted distinct sigma_e values of the problem's cells.
static std::vector<double> material_values(const slh_problem* p) {
  const long long n = (long long)p->nx * p->ny;
  std::vector<double> v(n);
  for (long long i = 0; i < n; ++i) v[i] = sigma_e_of(p, i);
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

// LDS bytes one workgroup may use on the current device.
static size_t lds_limit() {
  static std::mutex mu;  // solvers and servers are created from several threads
  static size_t cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  std::lock_guard<std::mutex> lk(mu);
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v < 65536)
      v = 65536;
    cached[dev] = (size_t)v;
  }
  return cached[dev];
}

// Chooses the sweep.  n_mat < 0: the fields are not known (footprint bound).
// Chunks of 1024 or 512 cells (four or two per lane: fewer barriers per
// sweep) where the diagonals are that long, else of up to 256 cells, one per
// lane; the table mode wherever its coefficients fit in LDS beside the chunk
// slots and the face traces, else the cell mode.
static void plan_dg(Sizes& z, const slh_problem* p, long long n_mat) {
  const int diag = std::min(p->nx, p->ny);  // longest diagonal
  std::vector<std::pair<int, int>> cand;    // (cells per lane, cells per chunk)
  for (int q = 4; q > 1; q /= 2)
    if (diag >= 256 * q) cand.emplace_back(q, 256 * q);
  for (int cw = std::min(256, (diag + 63) / 64 * 64); cw >= 64; cw -= 64) cand.emplace_back(1, cw);
  const size_t lim = lds_limit();
  z.n_mat = n_mat < 0 ? (int)std::max<long long>(0, (long long)(lim / 256)) : (int)n_mat;
  z.dg_q = 1;
  z.dg_cw = 64;  // nothing fits: set-up reports the mesh as too large
  z.dg_table = false;
  bool chosen = false;
  for (int table = n_mat > 0 ? 1 : 0; table >= 0 && !chosen; --table)
    for (const auto& c : cand)
      if ((table || c.first <= 2) &&  // four cell-mode solves per lane spill registers
          dg_sweep_lds_bytes(table != 0, c.second, table ? z.n_mat : 0, p->nx, p->ny) <= lim) {
        z.dg_q = c.first;
        z.dg_cw = c.second;
        z.dg_table = table != 0;
        chosen = true;
        break;
      }
  if (n_mat < 0) z.dg_table = true;  // bound: table storage counted
  z.dg_chunks = dg_chunks(p->nx, p->ny, z.dg_cw);
}

static bool finite_nonneg(const double* p, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!(p[i] >= 0.0) || !isfinite(p[i])) return false;
  return true;
}

static slh_status validate(const slh_problem* p, bool check_fields) {
  if (!p) return fail(SLH_E_INVALID_ARG, "problem is NULL");
  if (p->abi_version != SLH_ABI_VERSION) return fail(SLH_E_INVALID_ARG, "abi_version mismatch");
  if (p->nx < 1 || p->ny < 1) return fail(SLH_E_INVALID_ARG, "nx, ny must be >= 1");
  if ((long long)p->nx * p->ny > (1ll << 30)) return fail(SLH_E_INVALID_ARG, "mesh too large");
  if (p->nx + p->ny > 4096) return fail(SLH_E_INVALID_ARG, "nx + ny must be <= 4096");
  if (!(p->x_hi > p->x_lo) || !(p->y_hi > p->y_lo) || !isfinite(p->x_lo) || !isfinite(p->x_hi) ||
      !isfinite(p->y_lo) || !isfinite(p->y_hi))
    return fail(SLH_E_INVALID_ARG, "empty or non-finite domain");
  if (p->steady != 0 && p->steady != 1) return fail(SLH_E_INVALID_ARG, "steady must be 0 or 1");
  if (p->si_norm != SLH_SI_NORM_COLLIDED && p->si_norm != SLH_SI_NORM_TOTAL)
    return fail(SLH_E_INVALID_ARG, "si_norm must be SLH_SI_NORM_COLLIDED or SLH_SI_NORM_TOTAL");
  if (p->closure != SLH_CLOSE_SN && p->closure != SLH_CLOSE_DIFFUSION)
    return fail(SLH_E_INVALID_ARG, "closure must be SLH_CLOSE_SN or SLH_CLOSE_DIFFUSION");
  if (p->si_accel != SLH_ACCEL_NONE && p->si_accel != SLH_ACCEL_DSA)
    return fail(SLH_E_INVALID_ARG, "si_accel must be SLH_ACCEL_NONE or SLH_ACCEL_DSA");
  if (!p->steady) {
    if (!(p->c > 0.0) || !isfinite(p->c)) return fail(SLH_E_INVALID_ARG, "c must be > 0");
    if (!(p->dt > 0.0) || !isfinite(p->dt)) return fail(SLH_E_INVALID_ARG, "dt must be > 0");
  } else {
    if (!(p->horizon >= 0.0) || !isfinite(p->horizon))
      return fail(SLH_E_INVALID_ARG, "horizon must be finite and >= 0");
    if (p->horizon == 0.0 && !(p->w_cut_rel > 0.0 && p->w_cut_rel < 1.0))
      return fail(SLH_E_INVALID_ARG,
                  "steady state without a horizon needs 0 < w_cut_rel < 1 (default horizon)");
  }
  if (p->n_s < -1 || p->n_s > 1000000)
    return fail(SLH_E_INVALID_ARG, "n_s must be -1 (unlimited) or in [0, 1e6]");
  if (p->boundary < 0 || p->boundary > 15)
    return fail(SLH_E_INVALID_ARG, "boundary must be a mask of SLH_REFLECT_* (0..15)");
  if (check_fields && p->inflow) {
    const int nx = p->nx, ny = p->ny;
    for (int f = 0; f < 2 * (nx + ny); ++f) {
      int k;
      const int side = face_side(f, nx, ny, &k);
      const double g = p->inflow[f];
      if (!isfinite(g)) return fail(SLH_E_INVALID_ARG, "inflow values must be finite");
      if (g != 0.0 && (p->boundary & (1 << side)))
        return fail(SLH_E_INVALID_ARG, "inflow on a reflective side");
    }
  }
  if (check_fields && p->n_s_cell) {
    const long long n = (long long)p->nx * p->ny;
    for (long long i = 0; i < n; ++i)
      if (p->n_s_cell[i] < -1 || p->n_s_cell[i] > 1000000)
        return fail(SLH_E_INVALID_ARG, "n_s_cell entries must be -1 (unlimited) or in [0, 1e6]");
  }
  if (p->n_particles < 0 || p->n_particles > (1ll << 31))  // a cell's index l stays 32-bit
    return fail(SLH_E_INVALID_ARG, "n_particles must be in [0, 2^31]");
  if (p->census_cap < 0 || p->census_cap > (1ll << 31))
    return fail(SLH_E_INVALID_ARG, "census_cap out of range");
  {  // census slots are 32-bit: cap + source bank below 2^32
    const long long cap = p->census_cap > 0 ? p->census_cap : std::max<long long>(p->n_particles, 1);
    const long long src = p->n_particles + p->n_particles / 16 + (long long)p->nx * p->ny +
                          (p->inflow ? 2ll * (p->nx + p->ny) : 0) + 16;
    if (cap + src >= (1ll << 32))
      return fail(SLH_E_INVALID_ARG, "census cap plus source particles must stay below 2^32");
  }
  if (p->sn_order < 2 || p->sn_order % 2 || p->sn_order > 64)
    return fail(SLH_E_INVALID_ARG, "sn_order must be even in [2, 64]");
  if (!(p->time_closure >= 0.0) || !isfinite(p->time_closure))
    return fail(SLH_E_INVALID_ARG, "time_closure must be >= 0");
  if (!(p->si_tol >= 0.0) || !isfinite(p->si_tol)) return fail(SLH_E_INVALID_ARG, "si_tol < 0");
  if (p->si_max_iter < 0) return fail(SLH_E_INVALID_ARG, "si_max_iter < 0");
  if (p->census_qmc != SLH_CENSUS_HISTORY && p->census_qmc != SLH_CENSUS_COHORT)
    return fail(SLH_E_INVALID_ARG, "census_qmc must be 0 or 1");
  if (!(p->w_cut_rel >= 0.0) || !isfinite(p->w_cut_rel))
    return fail(SLH_E_INVALID_ARG, "w_cut_rel must be >= 0");
  if (p->points != SLH_SOBOL_OWEN && p->points != SLH_PRNG && p->points != SLH_HALTON)
    return fail(SLH_E_INVALID_ARG, "points must be SLH_SOBOL_OWEN, SLH_PRNG or SLH_HALTON");
  if (p->precision != SLH_FP64 && p->precision != SLH_FP32_TRACK)
    return fail(SLH_E_INVALID_ARG, "precision must be SLH_FP64 or SLH_FP32_TRACK");
  if (check_fields) {
    const long long n = (long long)p->nx * p->ny;
    if (!p->sigma_s || !p->sigma_a || !p->q) return fail(SLH_E_INVALID_ARG, "field is NULL");
    if (!finite_nonneg(p->sigma_s, n)) return fail(SLH_E_INVALID_ARG, "sigma_s must be finite, >= 0");
    if (!finite_nonneg(p->sigma_a, n)) return fail(SLH_E_INVALID_ARG, "sigma_a must be finite, >= 0");
    if (!finite_nonneg(p->q, n)) return fail(SLH_E_INVALID_ARG, "q must be finite, >= 0");
    if (p->steady && p->horizon == 0.0) {
      for (long long i = 0; i < n; ++i)
        if (!(p->sigma_a[i] > 0.0))
          return fail(SLH_E_INVALID_ARG,
                      "steady state with a cell of sigma_a = 0 needs an explicit horizon");
    }
    if (p->closure == SLH_CLOSE_DIFFUSION || p->si_accel == SLH_ACCEL_DSA)
      for (long long i = 0; i < n; ++i)
        if (!(p->sigma_a[i] + p->sigma_s[i] + time_term(p) > 0.0))
          return fail(SLH_E_INVALID_ARG, "the diffusion closure and the diffusion correction "
                                         "need sigma_t + tau/(c dt) > 0 in every cell");
    if (p->steady && !(horizon_of(p) <= 1e15))
      return fail(SLH_E_INVALID_ARG, "horizon above 1e15 (a small sigma_a sets the default)");
  }
  return SLH_OK;
}

static Sizes sizes_of(const slh_problem* p) {
  Sizes z;
  z.n_cells = (long long)p->nx * p->ny;
  z.n_p = p->n_particles;
  // the plan emits sum_i n_i < sum_i M_i / w_q + (emitters) particles, and
  // sum_i M_i / w_q < n_p (1 + 1/16), w_q being sum(M) / n_p rounded down to
  // five significant bits
  z.n_faces = p->inflow ? 2ll * (p->nx + p->ny) : 0;
  z.n_src_cap = z.n_p > 0 ? z.n_p + z.n_p / 16 + z.n_cells + z.n_faces + 16 : 0;
  z.cap = p->census_cap > 0 ? p->census_cap : std::max<long long>(p->n_particles, 1);
  z.n_cand = z.cap + z.n_src_cap;
  z.n_dir = p->sn_order * p->sn_order;
  // private tally copies: 16 per XCD on meshes of 64K cells or more (the
  // adds of a pass spread over more copies wait less on each other: on a
  // 1024^2 mesh 128 copies take each pass from 44 to 40 ms, where 32, 64 and
  // 256 copies do not), else 8 per XCD; halved while a tally array would
  // exceed 1 GB, down to one copy per XCD, then below
  z.n_copies = z.n_cells >= 65536 ? 128 : 64;
  while (z.n_copies > 1 &&
         (size_t)z.n_copies * kTallyStride * 8 * (size_t)z.n_cells > ((size_t)1 << 30))
    z.n_copies /= 2;
  z.fp32 = p->precision == SLH_FP32_TRACK;
  z.diffusion = p->closure == SLH_CLOSE_DIFFUSION;
  z.dsa = !z.diffusion && p->si_accel == SLH_ACCEL_DSA;
  const bool fields = p->sigma_s && p->sigma_a;
  plan_dg(z, p, fields ? (long long)material_values(p).size() : -1);
  if (fields) {
    const long long m = (long long)material_pairs(p).size();
    z.n_mc_mat = m <= kMaxMatIds ? (int)m : 0;
  } else {
    z.n_mc_mat = kMaxMatIds;  // bound
  }
  const size_t bank = z.fp32 ? sizeof(StageRec<float>) : sizeof(StageRec<double>);
  const size_t srec = z.fp32 ? sizeof(SrcRec<float>) : sizeof(SrcRec<double>);
  size_t b = 0;
  const size_t nc = (size_t)z.n_cells;
  b += nc * (16 + 8 + 8 + 16 + 8);           // mat64, mat32, sig_s, sig_e (two layouts), q
  if (z.n_mc_mat) b += nc * 2 + (size_t)z.n_mc_mat * 24;  // material ids and tables
  if (p->n_s_cell) b += nc * 4;              // per-cell scatter limits
  if (p->boundary)                           // mirror indices, reflected traces
    b += (size_t)z.n_dir * 8 + (size_t)2 * z.n_dir * 2 * (p->nx + p->ny) * 8;
  b += nc * 32 * 2 + (size_t)tree_leaves(z.n_cells + z.n_faces) * 16 * 2;  // sources, count trees
  b += (size_t)kMajGroups * kMajBins * 8;    // majorant histograms
  b += (size_t)z.n_faces * 8;                // inflow of the boundary faces
  b += nc * 8 * kTallyStride * 3 * (size_t)z.n_copies;  // tallies
  b += nc * 8 * 3 + nc * 32 * 3;             // phi_pre/post/R, phi_c, DG source x2
  b += (size_t)z.n_dir * 4;                  // directions of each sweep layout
  if (!z.diffusion) b += nc * 64;            // per-layout direction sums
  if (z.diffusion || z.dsa)
    b += nc * 8 * 9 + 4 * 1024 * 8;          // CG: diag, cE, cN, x, r, z, p x2, q; partials
  if (z.dsa) b += nc * 32;                   // nodal change of a sweep
  if (!z.diffusion) b += (size_t)z.n_dir * nc * 32;  // direction planes
  b += (size_t)z.n_dir * 256;                // element data
  if (z.dg_table) b += nc * 8 + (size_t)z.n_mat * 8 + (size_t)z.n_dir * z.n_mat * 256;
  b += (size_t)z.n_dir * 24 + 1024 * 16 + 4096;
  b += (size_t)z.cap * bank * 2;             // census banks
  b += (size_t)(z.n_src_cap > 0 ? z.n_src_cap : 1) * srec;  // source bank
  b += (size_t)z.n_cand * ((z.fp32 ? 32 : 64) + 1 + 4);  // staging, alive, kept cells
  b += (size_t)census_tiles(z.n_cand) * 16;          // tile counts and their scan
  b += std::max(scan_tmp_elems(census_tiles(z.n_cand)),
                scan_tmp_elems((long long)radix_hist_elems(z.cap))) * 8;
  b += (size_t)z.cap * 4 * 6 + radix_hist_elems(z.cap) * 16 + nc * 4;  // census ordering
  b += sizeof(DevState) + 32 * 32 * 4 + 64 * 8 + kCensusBlocks * 8;
  b += 64 * 1024;  // alignment of the ~30 device buffers
  z.bytes = b;
  return z;
}

extern "C" size_t slh_footprint_bytes(const slh_problem* p) {
  if (validate(p, false) != SLH_OK) return 0;
  return sizes_of(p).bytes;
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
struct BalStore {
  unsigned long long bal[2 * B_NFIELDS];
  unsigned long long segments, particles, alive, killed;
  double unit_W;
  long long n_in;
  long long n_emit;
  double sumM, wq;
  int thin_overflow;  // of the census that this pass read
  int numeric;        // DevState::numeric of the pass
};

// End of a pass: its balance record for slh_get_balance; at the end of the
// remap pass also the step's device totals (both passes: a step that halts
// between them books nothing, so running it again counts it once;
// si_active: the step had a source iteration, whose state is final then).
__global__ void k_snapshot(DevState* st, BalStore* out, int kind, int si_active) {
  if (st->halt) return;
  const int t = threadIdx.x;
  if (t < 2 * B_NFIELDS) out->bal[t] = st->bal[t];
  if (t == 0) {
    if (kind == 2) {
      const BalStore* p1 = out - 1;  // the pass-1 record of this step
      int num = p1->numeric | (p1->killed ? 16 : 0) | st->numeric | (st->killed ? 16 : 0);
      st->acc_seg[0] += p1->segments;
      st->acc_seg[1] += st->segments;
      st->acc_killed += p1->killed + st->killed;
      st->acc_census_in += (unsigned long long)p1->n_in;
      st->acc_thin_overflow += p1->thin_overflow ? 1ull : 0ull;
      st->acc_census_out += st->alive;
      st->acc_steps += 1ull;
      if (si_active && !st->si.conv) st->acc_unconv += 1ull;
      if (si_active && st->si.bad) num |= 8;
      st->acc_numeric |= num;
    }
    out->segments = st->segments;
    out->particles = st->particles;
    out->alive = st->alive;
    out->killed = st->killed;
    out->unit_W = st->unit_W;
    out->n_in = st->n_in;
    out->n_emit = st->n_emit;
    out->sumM = st->sumM[kind - 1];
    out->wq = st->wq[kind - 1];
    out->thin_overflow = st->thin_overflow;
    out->numeric = st->numeric;
  }
}

__global__ void k_state_init(DevState* st) {
  if (threadIdx.x == 0) {
    memset(st, 0, sizeof(DevState));
    st->thin_factor = 1.0;
  }
}

// A loaded checkpoint: its bank, its step, and fresh totals.
__global__ void k_state_set_bank(DevState* st, long long n, double maxabs,
                                 unsigned long long step) {
  if (threadIdx.x == 0) {
    st->halt = 0;
    st->step = step;
    st->n_in = n;
    st->n_kept = n;
    st->maxabs_w = maxabs;
    st->acc_seg[0] = st->acc_seg[1] = 0ull;
    st->acc_census_in = st->acc_census_out = st->acc_killed = st->acc_steps = 0ull;
    st->acc_thin_overflow = st->acc_unconv = 0ull;
    st->acc_numeric = 0;
  }
}

// HIP events of one step launched in timing mode: start, MC pass 1 start and
// end, end of the collided solve and remap set-up, MC pass 2 start and end,
// end of the step.
struct StepEvents {
  hipEvent_t e[7];
};

struct slh_solver {
  slh_problem prob;
  Sizes z;
  hipStream_t stream = nullptr;
  slh_alloc_fn alloc = nullptr;
  bool misaligned = false;  // the allocator returned memory not aligned to 256 bytes
  slh_free_fn free_fn = nullptr;
  void* ctx = nullptr;
  std::vector<void*> allocs;
  // static scratch (slh_create_static): device memory is carved from the
  // device's scratch array by a bump pointer; nothing is allocated or freed
  bool static_mem = false;
  int static_dev = -1;
  char* bump_base = nullptr;
  size_t bump_off = 0, bump_len = 0;
  std::vector<double> h_sig_s, h_sig_a, h_q;
  std::vector<int> h_ns;    // per-cell scatter limits (unlimited as INT_MAX), empty if uniform
  int n_lim_max = 0;        // the largest limit of the scatter-limited leg
  int* ns_cell = nullptr;   // device copy of h_ns
  double hx, hy, area, adt, tau, si_tol;
  double horizon = 0.0;     // steady state: path length at which a history ends
  bool skip_remap = false;  // steady pure MC: no collided solve, phi_R = phi_pre
  // diffusion closing stage: coefficients, CG vectors, block partials
  double* dnode = nullptr;  // diffusion correction: nodal change of a sweep
  double *cg_diag = nullptr, *cg_e = nullptr, *cg_n = nullptr, *cg_x = nullptr,
         *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr,
         *cg_part = nullptr;
  int cg_npart = 0;
  long long thin_margin = 0;
  int si_max;

  // device memory
  double2* mat64 = nullptr;
  float2* mat32 = nullptr;
  uint16_t* mat_id16 = nullptr;  // tracking: material id per cell, and its tables
  double2* mtab64 = nullptr;
  float2* mtab32 = nullptr;
  double *sig_s = nullptr, *sig_e = nullptr, *q = nullptr;
  double *qn1 = nullptr, *ctree1 = nullptr;  // nodal source and count tree of each pass
  double *qnR = nullptr, *ctreeR = nullptr;
  unsigned long long* maj_hist = nullptr;     // histograms of the emission plan
  double* inflow = nullptr;                   // inflow of the boundary faces, or none
  std::vector<double> h_inflow;
  long long tree_L = 1;
  unsigned long long *Tpre = nullptr, *Tpost = nullptr, *TR = nullptr;
  double *phi_pre = nullptr, *phi_post = nullptr, *phi_R = nullptr, *phi_c = nullptr;
  double *psi = nullptr, *dg_part = nullptr, *dirs = nullptr;
  double* cmax = nullptr;  // per-block max |w| of the census compaction
  // reflective sides: mirror indices of the directions and two buffers of
  // boundary outflow traces (null when every side is vacuum)
  int *refl_x = nullptr, *refl_y = nullptr;
  double* bnd = nullptr;
  std::vector<int> h_refl;
  double* dirmat = nullptr;  // DG element data per direction
  int* mat_id = nullptr;     // DG table mode: material of each cell (sweep layouts),
  double *sig_e_mat = nullptr, *coef = nullptr;  // its sigma_e, coefficients
  double* dg_src = nullptr;  // nodal source of a sweep (sweep layouts)
  int* fam_dirs = nullptr;   // directions of layout A, then of layout B
  int fam_n = 0;             // how many of them belong to layout A
  double* phi_fam = nullptr; // per-layout direction sums of the reduction
  int n_part = 1;
  void* bank_mem[2] = {nullptr, nullptr};
  void* stage_mem = nullptr;
  void* src_mem = nullptr;  // source bank of the current pass
  uint8_t* alive = nullptr;
  int32_t* kcell = nullptr;  // cell of each kept candidate
  long long *tcount = nullptr, *tincl = nullptr, *scan_i = nullptr;
  // census ordering: (cell, slot) pairs and their sort buffers, the radix
  // histograms, cohort starts per cell, and each bank's cohort ranks
  uint32_t *skey[2] = {nullptr, nullptr}, *sval[2] = {nullptr, nullptr};
  long long *rhist = nullptr, *rincl = nullptr;
  uint32_t* cstart = nullptr;
  uint32_t* crank[2] = {nullptr, nullptr};
  uint32_t* sobol = nullptr;
  DevState* st = nullptr;
  BalStore* bal_store = nullptr;  // [2]
  int cur = 0;

  // host-side state
  long long step = 0;             // steps enqueued
  // graphs: one per step and census-bank parity (production), or the three
  // graph parts of a step in timing mode, keyed by (part, parity)
  bool use_graphs = true;
  int grid1 = 1, grid2 = 1;       // persistent grids of the two MC passes
  bool timing = false;            // steps as graph parts and MC kernels between events
  hipStream_t cap_stream = nullptr;
  std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;  // (part, parity, batch)
  // source iterations launched per step: si_batch (adaptive) in production;
  // a step whose batch ends before the iteration halts itself and the steps
  // after it on the device, and settle() runs them again
  int si_batch = 0;
  unsigned long long last_halted = ~0ull;  // step index of the last halted step
  int batch_run = 0;          // the batch of the step being enqueued
  // conjugate-gradient steps launched per diffusion correction (adaptive, at
  // most kDsaMaxIter; a correction they leave unfinished halts its step)
  int cg_batch = 16;
  int cg_run = 0;
  bool unsettled = false;     // steps enqueued since the last settle()
  unsigned long long restarts = 0ull;  // steps run again after a halt
  unsigned long long graph_launches = 0ull;
  // timing mode: events of the steps enqueued since the last collection
  std::vector<StepEvents> ev_pool;
  size_t ev_used = 0;
  double k_ms[2] = {0.0, 0.0};    // MC-pass kernel times (timing mode)
  double stage_ms[4] = {0.0, 0.0, 0.0, 0.0};  // last timed step
  bool have_stage = false;
  // device totals already turned into a status by slh_synchronize
  unsigned long long rep_unconv = 0ull;
  int rep_numeric = 0;

  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 8;
    void* p = nullptr;
    if (static_mem) {
      const size_t off = (bump_off + 255) / 256 * 256;
      if (off + bytes > bump_len) return nullptr;
      bump_off = off + bytes;
      return bump_base + off;
    } else if (alloc) {
      p = alloc(bytes, ctx);
      if (p && ((uintptr_t)p & 255u)) {  // the kernels' vector loads need alignment
        if (free_fn) free_fn(p, ctx);
        misaligned = true;
        return nullptr;
      }
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
    if (p) allocs.push_back(p);
    return p;
  }
  void release() {
    for (auto& kv : graphs)
      if (kv.second) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    for (void* p : allocs) {
      if (free_fn) free_fn(p, ctx);
      else (void)hipFree(p);
    }
    allocs.clear();
    for (auto& se : ev_pool)
      for (auto& e : se.e)
        if (e) (void)hipEventDestroy(e);
    ev_pool.clear();
  }

  // census bank: an array of census records; source particles: an array of
  // source records (each record one piece of a cache line)
  size_t rec_bytes() const {
    return z.fp32 ? sizeof(StageRec<float>) : sizeof(StageRec<double>);
  }
  size_t bank_bytes(long long n) const { return (size_t)(n > 0 ? n : 1) * rec_bytes(); }
  size_t src_bytes(long long n) const {
    return (size_t)(n > 0 ? n : 1) * (z.fp32 ? sizeof(SrcRec<float>) : sizeof(SrcRec<double>));
  }
};

static slh_status setup(slh_solver* s) {
  const slh_problem& p = s->prob;
  const Sizes& z = s->z;
  const long long nc = z.n_cells;
#define ALLOC(ptr, T, n)                                                               \
  do {                                                                                 \
    ptr = (T*)s->dalloc(sizeof(T) * (size_t)(n));                                      \
    if (!ptr)                                                                          \
      return s->misaligned                                                             \
                 ? fail(SLH_E_INVALID_ARG, "the allocator returned memory not aligned "  \
                                           "to 256 bytes: " #ptr)                       \
                 : fail(SLH_E_OUT_OF_MEMORY, "device allocation failed: " #ptr);        \
  } while (0)
  if (dg_sweep_lds_bytes(false, z.dg_cw, 0, p.nx, p.ny) > lds_limit())
    return fail(SLH_E_INVALID_ARG, "nx + ny too large for the sweep's LDS traces");
  ALLOC(s->mat64, double2, nc);
  ALLOC(s->mat32, float2, nc);
  if (z.n_mc_mat) {
    ALLOC(s->mat_id16, uint16_t, nc);
    ALLOC(s->mtab64, double2, z.n_mc_mat);
    ALLOC(s->mtab32, float2, z.n_mc_mat);
  }
  ALLOC(s->sig_s, double, nc);
  ALLOC(s->sig_e, double, 2 * nc);  // sweep layouts A and B
  ALLOC(s->q, double, nc);
  if (!s->h_ns.empty()) ALLOC(s->ns_cell, int, nc);
  s->tree_L = tree_leaves(nc + z.n_faces);
  ALLOC(s->qn1, double, 4 * nc);
  ALLOC(s->ctree1, double, 2 * s->tree_L);
  ALLOC(s->qnR, double, 4 * nc);
  ALLOC(s->ctreeR, double, 2 * s->tree_L);
  ALLOC(s->maj_hist, unsigned long long, kMajGroups * kMajBins);
  if (z.n_faces) ALLOC(s->inflow, double, z.n_faces);
  ALLOC(s->Tpre, unsigned long long, (size_t)z.n_copies * kTallyStride * nc);
  ALLOC(s->Tpost, unsigned long long, (size_t)z.n_copies * kTallyStride * nc);
  ALLOC(s->TR, unsigned long long, (size_t)z.n_copies * kTallyStride * nc);
  ALLOC(s->phi_pre, double, nc);
  ALLOC(s->phi_post, double, nc);
  ALLOC(s->phi_R, double, nc);
  ALLOC(s->phi_c, double, 4 * nc);
  if (z.dsa) ALLOC(s->dnode, double, 4 * nc);
  if (!z.diffusion) ALLOC(s->psi, double, (size_t)z.n_dir * 4 * nc);
  if (z.diffusion || z.dsa) {
    ALLOC(s->cg_diag, double, nc);
    ALLOC(s->cg_e, double, nc);
    ALLOC(s->cg_n, double, nc);
    ALLOC(s->cg_x, double, nc);
    ALLOC(s->cg_r, double, nc);
    ALLOC(s->cg_z, double, nc);
    ALLOC(s->cg_p, double, 2 * nc);
    ALLOC(s->cg_q, double, nc);
    s->cg_npart = cg_partials(nc);
    ALLOC(s->cg_part, double, 4 * s->cg_npart);
  }
  ALLOC(s->dirmat, double, (size_t)z.n_dir * 32);
  if (z.dg_table) {
    ALLOC(s->mat_id, int, 2 * nc);
    ALLOC(s->sig_e_mat, double, z.n_mat);
    ALLOC(s->coef, double, (size_t)z.n_dir * z.n_mat * 32);
  }
  ALLOC(s->dg_src, double, 8 * nc);
  ALLOC(s->fam_dirs, int, z.n_dir);
  if (!z.diffusion) ALLOC(s->phi_fam, double, 8 * nc);
  s->n_part = dg_reduce_partials(4 * nc);
  ALLOC(s->dg_part, double, 2 * s->n_part + 2);
  ALLOC(s->cmax, double, kCensusBlocks);
  if (p.boundary) {
    ALLOC(s->refl_x, int, z.n_dir);
    ALLOC(s->refl_y, int, z.n_dir);
    ALLOC(s->bnd, double, (size_t)2 * z.n_dir * 2 * (p.nx + p.ny));
  }
  ALLOC(s->dirs, double, 3 * z.n_dir);
  s->bank_mem[0] = s->dalloc(s->bank_bytes(z.cap));
  s->bank_mem[1] = s->dalloc(s->bank_bytes(z.cap));
  s->stage_mem = s->dalloc((size_t)z.n_cand * (z.fp32 ? sizeof(StageRec<float>)
                                                     : sizeof(StageRec<double>)));
  s->src_mem = s->dalloc(s->src_bytes(z.n_src_cap));
  if (!s->bank_mem[0] || !s->bank_mem[1] || !s->stage_mem || !s->src_mem)
    return s->misaligned ? fail(SLH_E_INVALID_ARG,
                                "the allocator returned memory not aligned to 256 bytes: banks")
                         : fail(SLH_E_OUT_OF_MEMORY, "device allocation failed: census banks");
  ALLOC(s->alive, uint8_t, z.n_cand);
  ALLOC(s->kcell, int32_t, z.n_cand);
  ALLOC(s->tcount, long long, census_tiles(z.n_cand));
  ALLOC(s->tincl, long long, census_tiles(z.n_cand));
  ALLOC(s->scan_i, long long, std::max(scan_tmp_elems(census_tiles(z.n_cand)),
                                      scan_tmp_elems((long long)radix_hist_elems(z.cap))));
  for (int k = 0; k < 2; ++k) {
    ALLOC(s->skey[k], uint32_t, z.cap);
    ALLOC(s->sval[k], uint32_t, z.cap);
    ALLOC(s->crank[k], uint32_t, z.cap);
  }
  ALLOC(s->rhist, long long, radix_hist_elems(z.cap));
  ALLOC(s->rincl, long long, radix_hist_elems(z.cap));
  ALLOC(s->cstart, uint32_t, nc);
  ALLOC(s->sobol, uint32_t, 32 * 32);
  ALLOC(s->st, DevState, 1);
  ALLOC(s->bal_store, BalStore, 2);
#undef ALLOC
  // fields and derived arrays
  std::vector<double2> m64(nc);
  std::vector<float2> m32(nc);
  std::vector<double> se(nc), qn(4 * nc);
  for (long long i = 0; i < nc; ++i) {
    m64[i] = make_double2(s->h_sig_s[i], s->h_sig_a[i]);
    m32[i] = make_float2((float)s->h_sig_s[i], (float)s->h_sig_a[i]);
    se[i] = s->h_sig_a[i] + s->h_sig_s[i] + time_term(&p);
    for (int k = 0; k < 4; ++k) qn[4 * i + k] = s->h_q[i];
  }
  const std::vector<double> dirs = product_quadrature(p.sn_order);
  hipStream_t st = s->stream;
  HIP_TRY(hipMemcpyAsync(s->mat64, m64.data(), sizeof(double2) * nc, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->mat32, m32.data(), sizeof(float2) * nc, hipMemcpyHostToDevice, st));
  std::vector<uint16_t> mid16;
  std::vector<double2> t64;
  std::vector<float2> t32;
  if (z.n_mc_mat) {
    std::vector<std::pair<double, double>> pairs;
    pairs.reserve(nc);
    for (long long i = 0; i < nc; ++i) pairs.emplace_back(s->h_sig_s[i], s->h_sig_a[i]);
    std::vector<std::pair<double, double>> uniq(pairs);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    if ((long long)uniq.size() != z.n_mc_mat) return fail(SLH_E_STATE, "material count changed");
    mid16.resize(nc);
    for (long long i = 0; i < nc; ++i)
      mid16[i] = (uint16_t)(std::lower_bound(uniq.begin(), uniq.end(), pairs[i]) - uniq.begin());
    for (const auto& u : uniq) {
      t64.push_back(make_double2(u.first, u.second));
      t32.push_back(make_float2((float)u.first, (float)u.second));
    }
    HIP_TRY(hipMemcpyAsync(s->mat_id16, mid16.data(), 2 * nc, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->mtab64, t64.data(), sizeof(double2) * t64.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->mtab32, t32.data(), sizeof(float2) * t32.size(),
                           hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(s->sig_s, s->h_sig_s.data(), 8 * nc, hipMemcpyHostToDevice, st));
  // sweep layouts: sigma_e in layouts A and B, and the directions of each
  // layout (A: both components of one sign)
  std::vector<double> se_l(2 * nc);
  for (long long c = 0; c < nc; ++c) {
    const int ci = (int)(c % p.nx), cj = (int)(c / p.nx);
    se_l[lay_pos(p.nx, p.ny, ci, cj, true)] = se[c];
    se_l[nc + lay_pos(p.nx, p.ny, ci, cj, false)] = se[c];
  }
  std::vector<int> fam;
  for (int f = 0; f < 2; ++f)
    for (int m = 0; m < z.n_dir; ++m)
      if (((dirs[3 * m] > 0.0) == (dirs[3 * m + 1] > 0.0)) == (f == 0)) fam.push_back(m);
  s->fam_n = 0;
  for (int m = 0; m < z.n_dir; ++m)
    if ((dirs[3 * m] > 0.0) == (dirs[3 * m + 1] > 0.0)) s->fam_n += 1;
  HIP_TRY(hipMemcpyAsync(s->sig_e, se_l.data(), 16 * nc, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->fam_dirs, fam.data(), 4 * fam.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->q, s->h_q.data(), 8 * nc, hipMemcpyHostToDevice, st));
  if (s->ns_cell)
    HIP_TRY(hipMemcpyAsync(s->ns_cell, s->h_ns.data(), 4 * nc, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->qn1, qn.data(), 32 * nc, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->dirs, dirs.data(), 8 * dirs.size(), hipMemcpyHostToDevice, st));
  if (p.boundary) {
    // mirror image of each direction in x (Ox -> -Ox) and in y (Oy -> -Oy):
    // the product set is symmetric, so the nearest direction is exact
    const int nd = z.n_dir;
    s->h_refl.assign(2 * nd, 0);
    for (int m = 0; m < nd; ++m) {
      double bx = 1e300, by = 1e300;
      for (int k = 0; k < nd; ++k) {
        const double ex = fabs(dirs[3 * k] + dirs[3 * m]) + fabs(dirs[3 * k + 1] - dirs[3 * m + 1]);
        const double ey = fabs(dirs[3 * k] - dirs[3 * m]) + fabs(dirs[3 * k + 1] + dirs[3 * m + 1]);
        if (ex < bx) { bx = ex; s->h_refl[m] = k; }
        if (ey < by) { by = ey; s->h_refl[nd + m] = k; }
      }
    }
    HIP_TRY(hipMemcpyAsync(s->refl_x, s->h_refl.data(), 4 * nd, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->refl_y, s->h_refl.data() + nd, 4 * nd, hipMemcpyHostToDevice, st));
  }
  std::vector<int> mid;
  std::vector<double> mval;
  if (z.dg_table) {
    mval.assign(se.begin(), se.end());
    std::sort(mval.begin(), mval.end());
    mval.erase(std::unique(mval.begin(), mval.end()), mval.end());
    if ((long long)mval.size() != z.n_mat) return fail(SLH_E_STATE, "material count changed");
    mid.resize(2 * nc);
    for (long long c = 0; c < nc; ++c) {
      const int k = (int)(std::lower_bound(mval.begin(), mval.end(), se[c]) - mval.begin());
      const int ci = (int)(c % p.nx), cj = (int)(c / p.nx);
      mid[lay_pos(p.nx, p.ny, ci, cj, true)] = k;
      mid[nc + lay_pos(p.nx, p.ny, ci, cj, false)] = k;
    }
    HIP_TRY(hipMemcpyAsync(s->mat_id, mid.data(), 8 * nc, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->sig_e_mat, mval.data(), 8 * z.n_mat, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(launch_dg_tables(z.n_dir, z.dg_table ? z.n_mat : 0, s->dirs, s->sig_e_mat, s->hx,
                           s->hy, s->dirmat, s->coef, st));
  // the diffusion correction takes the vacuum condition on every side (the
  // sweep's reflected inflow lags one iteration; a zero-current side there
  // makes the corrected iteration diverge)
  if (z.diffusion || z.dsa)
    HIP_TRY(launch_diff_coef(p.nx, p.ny, s->mat64, time_term(&p), s->hx, s->hy,
                             z.dsa ? 0 : p.boundary, s->cg_diag, s->cg_e, s->cg_n, st));
  HIP_TRY(hipMemcpyAsync(s->sobol, sobol_table_host(), 4 * 32 * 32, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_fill_u64(s->maj_hist, kMajGroups * kMajBins, 0ull, st));  // left zero by every plan
  if (z.n_faces)
    HIP_TRY(hipMemcpyAsync(s->inflow, s->h_inflow.data(), 8 * z.n_faces, hipMemcpyHostToDevice,
                           st));
  HIP_TRY(launch_fill_f64(s->ctree1, 2 * s->tree_L, 0.0, st));
  HIP_TRY(launch_fill_f64(s->ctreeR, 2 * s->tree_L, 0.0, st));
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, st, s->st);
  HIP_TRY(launch_fill_f64(s->phi_c, 4 * nc, 0.0, st));
  HIP_TRY(launch_fill_f64(s->phi_pre, nc, 0.0, st));
  HIP_TRY(launch_fill_f64(s->phi_post, nc, 0.0, st));
  HIP_TRY(launch_fill_f64(s->phi_R, nc, 0.0, st));
  HIP_TRY(launch_fill_u64((unsigned long long*)s->bal_store, 2 * sizeof(BalStore) / 8, 0ull, st));
  HIP_TRY(launch_fill_u8(s->alive, z.n_cand, 0, st));
  HIP_TRY(hipStreamSynchronize(st));  // host vectors above go out of scope
  return SLH_OK;
}

// The boundary faces of the inflow as emitters after the cells: face f's
// majorant is (pi L_f) tdt pow2_ceil(|G_f|), the partial current pi G of an
// isotropic inflow over the face and the step (tdt = 1 in steady state).
static Emitters emitters(const slh_solver* s) {
  Emitters e;
  e.inflow = s->inflow;
  e.nx = s->prob.nx;
  e.ny = s->prob.ny;
  e.n_faces = s->z.n_faces;
  const double tdt = s->prob.steady ? 1.0 : s->prob.dt;
  e.cx = (M_PI * s->hy) * tdt;
  e.cy = (M_PI * s->hx) * tdt;
  return e;
}

static PassArgs pass_args(slh_solver* s, int kind) {
  PassArgs a;
  memset(&a, 0, sizeof(a));
  const slh_problem& p = s->prob;
  a.nx = p.nx;
  a.ny = p.ny;
  a.hx = s->hx;
  a.hy = s->hy;
  // steady state: the census of the time-dependent step becomes the path
  // horizon (c = 1, dt = horizon), every particle starts at time 0, and no
  // census is kept
  a.dt = p.steady ? s->horizon : p.dt;
  a.c = p.steady ? 1.0 : p.c;
  a.dt_birth = p.steady ? 0.0 : p.dt;
  a.keep_census = p.steady ? 0 : 1;
  a.mat64 = s->mat64;
  a.mat32 = s->mat32;
  a.mat_id16 = s->mat_id16;
  a.mtab64 = s->mtab64;
  a.mtab32 = s->mtab32;
  a.ctree = kind == 1 ? s->ctree1 : s->ctreeR;
  a.adt = s->adt;
  a.tree_L = s->tree_L;
  a.qn = kind == 1 ? s->qn1 : s->qnR;
  a.n_cells = s->z.n_cells;
  a.n_src = s->z.n_p;
  a.src_cap = s->z.n_src_cap;
  a.seed = p.seed;
  a.kind = kind;
  // n_s = -1: no scatter limit (the leg is plain implicit-capture MC)
  a.n_lim = kind == 1 ? s->n_lim_max : 0;
  a.ns_cell = kind == 1 ? s->ns_cell : nullptr;
  a.bc = p.boundary;
  a.points = p.points;
  a.sobol = s->sobol;
  a.w_cut_rel = p.w_cut_rel;
  a.max_segments = 1u << 26;
  void* bin = s->bank_mem[s->cur];
  a.in_rank = s->crank[s->cur];
  a.em = emitters(s);
  a.census_qmc = p.census_qmc;
  if (s->z.fp32) {
    a.in32 = (const StageRec<float>*)bin;
    a.out32 = (StageRec<float>*)s->stage_mem;
    a.src32 = (SrcRec<float>*)s->src_mem;
  } else {
    a.in64 = (const StageRec<double>*)bin;
    a.out64 = (StageRec<double>*)s->stage_mem;
    a.src64 = (SrcRec<double>*)s->src_mem;
  }
  a.alive = s->alive;
  a.out_src_base = s->z.cap;
  a.Ta = kind == 1 ? s->Tpre : s->TR;
  a.Tb = kind == 1 ? s->Tpost : s->TR;
  a.n_copies = s->z.n_copies;
  a.xcd_local = s->z.n_copies % kNumXcd == 0 ? 1 : 0;
  a.copy_stride = (long long)kTallyStride * s->z.n_cells;
  a.st = s->st;
  return a;
}

// A time step is five parts, enqueued in this order on the solver's stream:
//   kA    emission plan, pass set-up and emission of the scatter-limited leg
//   kMC1  MC pass 1
//   kMid  tally -> flux, pass-1 snapshot, phi_c = 0 and the source iteration
//         of the collided solve: si_max iterations, each returning at once
//         once the device's stopping test has said done; then the remap
//         source, its emission plan, pass set-up and emission
//   kMC2  MC pass 2 (the remap)
//   kEnd  tally -> flux, snapshot, census thinning and compaction, step + 1
// Every kernel reads its step-dependent values (step counter, counts, flags,
// the iteration state) from the device, so nothing in a step waits for the
// host.  In production the five parts are one graph, captured once per
// census-bank parity and replayed for every step; in timing mode kA, kMid and
// kEnd are graphs and the MC passes are launched between HIP events; with
// graphs off every kernel is launched directly.  All three give the same
// results.
enum Part { kA = 0, kMC1, kMid, kMC2, kEnd, kNumParts, kWhole = 9 };

static DgArgs dg_args(slh_solver* s) {
  const slh_problem& p = s->prob;
  const Sizes& z = s->z;
  DgArgs d;
  d.nx = p.nx;
  d.ny = p.ny;
  d.hx = s->hx;
  d.hy = s->hy;
  d.n_dir = z.n_dir;
  d.dir = s->dirs;
  d.fam_dirs = s->fam_dirs;
  d.fam_n = s->fam_n;
  d.sig_e = s->sig_e;
  d.sig_s = s->sig_s;
  d.phi_post = s->phi_post;
  d.phi_pre = s->prob.si_norm == SLH_SI_NORM_TOTAL ? s->phi_pre : nullptr;
  d.phi_c = s->phi_c;
  d.src = s->dg_src;
  d.psi = s->psi;
  d.phi_fam = s->phi_fam;
  d.dnode = s->z.dsa && !s->skip_remap ? s->dnode : nullptr;
  d.mat_id = s->mat_id;
  d.n_mat = z.n_mat;
  d.cw = z.dg_cw;
  d.coef = s->coef;
  d.dirmat = s->dirmat;
  d.n_chunks = (int)z.dg_chunks;
  d.cells_per_lane = z.dg_q;
  d.bc = s->prob.boundary;
  d.refl_x = s->refl_x;
  d.refl_y = s->refl_y;
  d.bnd = s->bnd;
  d.st = s->st;
  return d;
}

static CgArgs cg_args(slh_solver* s) {
  CgArgs c;
  c.nx = s->prob.nx;
  c.ny = s->prob.ny;
  c.diag = s->cg_diag;
  c.cE = s->cg_e;
  c.cN = s->cg_n;
  c.x = s->cg_x;
  c.r = s->cg_r;
  c.z = s->cg_z;
  c.P = s->cg_p;
  c.q = s->cg_q;
  c.n_part = s->cg_npart;
  c.part_a = s->cg_part;
  c.part_b = s->cg_part + 2 * s->cg_npart;
  // the closing stage's solve is the step's iteration; the correction is a
  // solve inside each source iteration, skipped once that iteration is done
  c.cs = s->z.diffusion ? &s->st->si : &s->st->dsa;
  c.gate = s->z.diffusion ? nullptr : &s->st->si.done;
  return c;
}

// Diffusion correction of a source iteration: tolerance and iteration limit
// of its conjugate gradients.  A loose solve is enough for the correction
// (its fixed point is the plain iteration's), and the fixed limit lets a
// batch of source iterations launch each correction's iterations blindly.
constexpr double kDsaTol = 1e-2;
constexpr int kDsaMaxIter = 32;

// the collided solve proper: the diffusion closing stage unless the step
// has no collided solve at all
static bool use_cg(const slh_solver* s) { return s->z.diffusion && !s->skip_remap; }

static slh_status enqueue_si(slh_solver* s, hipStream_t st, int n_it) {
  const Sizes& z = s->z;
  if (use_cg(s)) {
    const CgArgs c = cg_args(s);
    for (int it = 0; it < n_it; ++it) HIP_TRY(launch_cg_iteration(c, s->si_tol, s->si_max, st));
  } else if (z.dsa && !s->skip_remap) {
    const DgArgs d = dg_args(s);
    const CgArgs c = cg_args(s);
    for (int it = 0; it < n_it; ++it) {
      HIP_TRY(launch_dg_sweep(d, z.dg_table, st));
      HIP_TRY(launch_dg_reduce(d, s->dg_part, s->n_part, s->si_tol, s->si_max, st));
      HIP_TRY(launch_dsa_start(c, s->sig_s, s->dnode, kDsaMaxIter, st));
      if (cg_one_block(z.n_cells)) {
        HIP_TRY(launch_cg_solve_one_block(c, kDsaTol, kDsaMaxIter, st));
      } else {  // steps past convergence return at once
        for (int k = 0; k < s->cg_run; ++k)
          HIP_TRY(launch_cg_iteration(c, kDsaTol, kDsaMaxIter, st));
        if (s->cg_run < kDsaMaxIter) HIP_TRY(launch_dsa_check(s->st, st));
      }
      HIP_TRY(launch_dsa_apply(d, s->cg_x, s->dg_part, s->n_part, s->si_tol, s->si_max, st));
    }
  } else {
    const DgArgs d = dg_args(s);
    for (int it = 0; it < n_it; ++it) {
      HIP_TRY(launch_dg_sweep(d, z.dg_table, st));
      HIP_TRY(launch_dg_reduce(d, s->dg_part, s->n_part, s->si_tol, s->si_max, st));
    }
  }
  return SLH_OK;
}

static slh_status enqueue_part(slh_solver* s, int part, hipStream_t st) {
  const slh_problem& p = s->prob;
  const Sizes& z = s->z;
  const long long nc = z.n_cells;
  const double inv_adt = 1.0 / s->adt;
  const double cdt = p.steady ? s->horizon : p.c * p.dt;  // longest path of a history
  const long long cstride = (long long)kTallyStride * nc;
  const long long n_tally = (long long)z.n_copies * kTallyStride * nc;
  // source iterations launched in this step's batch (each predicated on the
  // device's stopping test), none without a collided solve
  const int n_it = s->skip_remap ? 0 : s->batch_run;
  switch (part) {
    case kA: {
      HIP_TRY(launch_emission_plan(s->qn1, nc, emitters(s), s->adt, z.n_p, p.seed, p.points, 1,
                                   s->maj_hist,
                                   s->ctree1, s->st, st));
      HIP_TRY(launch_pass_prep(s->st, s->ctree1, 1, z.n_src_cap, cdt, s->Tpre, n_tally, s->Tpost,
                               n_tally, nullptr, 0, st));
      HIP_TRY(launch_emit(pass_args(s, 1), z.fp32, st));
      return SLH_OK;
    }
    case kMC1:
      HIP_TRY(launch_mc_pass(pass_args(s, 1), z.fp32, s->grid1, st));
      return SLH_OK;
    case kMid: {
      HIP_TRY(launch_tally_to_flux(s->Tpre, s->phi_pre, s->Tpost, s->phi_post, nc, z.n_copies,
                                   cstride, s->st, inv_adt, st));
      hipLaunchKernelGGL(k_snapshot, dim3(1), dim3(64), 0, st, s->st, s->bal_store + 0, 1, 0);
      if (use_cg(s)) {
        HIP_TRY(launch_cg_start(cg_args(s), s->sig_s, s->phi_post, s->si_max, &s->st->halt, st));
      } else {
        // pure MC in steady state: no collided solve (phi_c = 0, no sweep)
        HIP_TRY(launch_si_start(dg_args(s), s->skip_remap ? 0 : s->si_max, st));
      }
      {
        const slh_status r = enqueue_si(s, st, n_it);
        if (r != SLH_OK) return r;
      }
      // a batch short of the limit may end before the iteration does
      if (n_it > 0 && n_it < s->si_max) HIP_TRY(launch_si_check(s->st, st));
      if (s->skip_remap) {  // no remap leg: clear its balance and census flags only
        HIP_TRY(launch_pass_prep(s->st, s->ctree1, 1, z.n_src_cap, cdt, nullptr, 0, nullptr, 0,
                                 s->alive, z.n_cand, st));
        return SLH_OK;
      }
      if (use_cg(s)) HIP_TRY(launch_cg_to_nodal(cg_args(s), s->phi_c, &s->st->halt, st));
      HIP_TRY(launch_remap_source(nc, s->q, s->sig_s, s->phi_pre, s->phi_post, s->phi_c,
                                  s->qnR, &s->st->halt, st));
      HIP_TRY(launch_emission_plan(s->qnR, nc, emitters(s), s->adt, z.n_p, p.seed, p.points, 2,
                                   s->maj_hist,
                                   s->ctreeR, s->st, st));
      HIP_TRY(launch_pass_prep(s->st, s->ctreeR, 2, z.n_src_cap, cdt, s->TR, n_tally, nullptr, 0,
                               s->alive, z.n_cand, st));
      HIP_TRY(launch_emit(pass_args(s, 2), z.fp32, st));
      return SLH_OK;
    }
    case kMC2:
      if (!s->skip_remap) HIP_TRY(launch_mc_pass(pass_args(s, 2), z.fp32, s->grid2, st));
      return SLH_OK;
    default: {  // kEnd: the remap census is the state at t_{n+1} (capped)
      // without a remap leg the solution is the pure-MC flux of pass 1
      HIP_TRY(launch_tally_to_flux(s->skip_remap ? s->Tpre : s->TR, s->phi_R, nullptr, nullptr,
                                   nc, z.n_copies, cstride, s->st, inv_adt, st));
      hipLaunchKernelGGL(k_snapshot, dim3(1), dim3(64), 0, st, s->st, s->bal_store + 1, 2,
                         n_it > 0 ? 1 : 0);
      void* nb = s->bank_mem[1 - s->cur];
      HIP_TRY(launch_thin_params(s->st, z.cap, s->thin_margin, st));
      // kept candidates (first cap in slot order), ordered by cell: the
      // census cohorts of the next step
      const long long tiles = census_tiles(z.n_cand);
      const long long* last = s->tincl + (tiles - 1);
      const int odd = radix_passes(nc) & 1;  // the sorted pairs end in buffer odd
      if (z.fp32)
        HIP_TRY(launch_census_keep(s->alive, (const StageRec<float>*)s->stage_mem, z.n_cand,
                                   p.seed, s->st, s->tcount, s->kcell, st));
      else
        HIP_TRY(launch_census_keep(s->alive, (const StageRec<double>*)s->stage_mem, z.n_cand,
                                   p.seed, s->st, s->tcount, s->kcell, st));
      HIP_TRY(scan_inclusive_i64(s->tcount, s->tincl, tiles, s->scan_i, &s->st->halt, st));
      HIP_TRY(launch_census_keys(s->kcell, s->alive, s->tcount, s->tincl, z.n_cand, z.cap,
                                 s->skey[0], s->sval[0], s->st, st));
      HIP_TRY(radix_sort_pairs(s->skey[0], s->sval[0], s->skey[1], s->sval[1], last, z.cap, nc,
                               s->rhist, s->rincl, s->scan_i, s->st, st));
      if (z.fp32)
        HIP_TRY(launch_census_gather<float>((const StageRec<float>*)s->stage_mem, s->sval[odd],
                                            last, z.cap, (StageRec<float>*)nb, s->st, s->cmax,
                                            st));
      else
        HIP_TRY(launch_census_gather<double>((const StageRec<double>*)s->stage_mem,
                                             s->sval[odd], last, z.cap, (StageRec<double>*)nb,
                                             s->st, s->cmax, st));
      HIP_TRY(launch_census_finish(s->st, s->tincl, tiles, z.cap, s->cmax, st));
      HIP_TRY(launch_cohort_ranks(s->skey[odd], &s->st->n_in, z.cap, s->cstart,
                                  s->crank[1 - s->cur], s->st, st));
      return SLH_OK;
    }
  }
}

// Parts [first, last] of a step on stream st.
static slh_status enqueue_parts(slh_solver* s, int first, int last, hipStream_t st) {
  for (int part = first; part <= last; ++part) {
    const slh_status r = enqueue_part(s, part, st);
    if (r != SLH_OK) return r;
  }
  return SLH_OK;
}

// Captures parts [first, last] on the capture stream.  Returns false when the
// runtime declines the capture; the solver then launches its kernels directly.
static bool capture(slh_solver* s, int first, int last, hipGraphExec_t* out) {
  *out = nullptr;
  if (!s->cap_stream &&
      hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    s->cap_stream = nullptr;
    return false;
  }
  if (hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return false;
  const slh_status r = enqueue_parts(s, first, last, s->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
  bool ok = r == SLH_OK && e == hipSuccess && g;
  if (ok) ok = hipGraphInstantiate(out, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  if (!ok) *out = nullptr;
  return ok;
}

// Parts [first, last] as one graph (key: first part, or kWhole for the whole
// step, and the census-bank parity), or directly.
static slh_status launch_parts(slh_solver* s, int first, int last, int key) {
  if (s->use_graphs) {
    const auto k = std::make_tuple(key, s->cur, s->batch_run * 64 + s->cg_run);
    auto it = s->graphs.find(k);
    if (it == s->graphs.end()) {
      hipGraphExec_t e = nullptr;
      if (capture(s, first, last, &e)) it = s->graphs.emplace(k, e).first;
      else s->use_graphs = false;
    }
    if (s->use_graphs) {
      HIP_TRY(hipGraphLaunch(it->second, s->stream));
      s->graph_launches += 1;
      return SLH_OK;
    }
  }
  return enqueue_parts(s, first, last, s->stream);
}

static slh_status record(hipEvent_t e, hipStream_t st) {
  HIP_TRY(hipEventRecord(e, st));
  return SLH_OK;
}

// Enqueues one time step with a batch of `batch` source iterations; no host
// wait.
static slh_status run_step(slh_solver* s, int batch) {
  slh_status r;
  s->batch_run = batch;
  s->cg_run = s->cg_batch;
  s->unsettled = true;
  if (!s->timing) {
    r = launch_parts(s, kA, kEnd, kWhole);
    if (r != SLH_OK) return r;
  } else {
    if (s->ev_used == s->ev_pool.size()) {
      StepEvents se;
      for (auto& e : se.e) e = nullptr;
      for (auto& e : se.e)
        if (hipEventCreate(&e) != hipSuccess) {
          for (auto& f : se.e)
            if (f) (void)hipEventDestroy(f);
          return fail(SLH_E_DEVICE, "hipEventCreate failed");
        }
      s->ev_pool.push_back(se);
    }
    const StepEvents& ev = s->ev_pool[s->ev_used++];
    hipStream_t st = s->stream;
    if ((r = record(ev.e[0], st)) != SLH_OK) return r;
    if ((r = launch_parts(s, kA, kA, kA)) != SLH_OK) return r;
    if ((r = record(ev.e[1], st)) != SLH_OK) return r;
    if ((r = enqueue_part(s, kMC1, st)) != SLH_OK) return r;
    if ((r = record(ev.e[2], st)) != SLH_OK) return r;
    if ((r = launch_parts(s, kMid, kMid, kMid)) != SLH_OK) return r;
    if ((r = record(ev.e[3], st)) != SLH_OK) return r;
    if ((r = enqueue_part(s, kMC2, st)) != SLH_OK) return r;
    if ((r = record(ev.e[4], st)) != SLH_OK) return r;
    if ((r = launch_parts(s, kEnd, kEnd, kEnd)) != SLH_OK) return r;
    if ((r = record(ev.e[5], st)) != SLH_OK) return r;
    if ((r = record(ev.e[6], st)) != SLH_OK) return r;
  }
  s->cur = 1 - s->cur;
  s->step += 1;
  return SLH_OK;
}

// After a stream synchronisation: folds the events of the timed steps into
// the kernel totals and keeps the stage times of the last one.
static slh_status collect_events(slh_solver* s) {
  for (size_t k = 0; k < s->ev_used; ++k) {
    const StepEvents& ev = s->ev_pool[k];
    float t[6];
    for (int i = 0; i < 6; ++i) HIP_TRY(hipEventElapsedTime(&t[i], ev.e[i], ev.e[i + 1]));
    s->k_ms[0] += t[1];
    s->k_ms[1] += t[3];
    s->stage_ms[0] = t[0] + t[1];  // emission and MC pass 1
    s->stage_ms[1] = t[2];         // collided solve and remap set-up
    s->stage_ms[2] = t[3];         // remap pass
    s->stage_ms[3] = t[4] + t[5];  // census
    s->have_stage = true;
  }
  s->ev_used = 0;
  return SLH_OK;
}

// ---------------------------------------------------------------------------
// Static scratch for callers that cannot allocate device memory (under graph
// capture, in serving loops, in harnesses that forbid it): slh_create_static
// carves a solver out of this array instead of calling an allocator.  Each
// device holds its own copy for the life of the process; host code must use
// the address hipGetSymbolAddress returns on that device, never the array's
// name.  One static solver may live on a device at a time.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {nullptr};
bool g_scratch_busy[kMaxDevices] = {false};
}  // namespace

// Device address of the current device's scratch (looked up once per
// device), reserved for one solver.
static slh_status scratch_acquire(int* dev_out, char** ptr_out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SLH_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_busy[dev])
    return fail(SLH_E_STATE, "the device's static scratch already holds a solver");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SLH_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  g_scratch_busy[dev] = true;
  *dev_out = dev;
  *ptr_out = g_scratch_ptr[dev];
  return SLH_OK;
}

static void scratch_release(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev >= 0 && dev < kMaxDevices) g_scratch_busy[dev] = false;
}

// A batch of source iterations: n rounded up to a multiple of four, at most
// the limit (fewer distinct batches, fewer captured graphs).
static int round_batch(long long n, int si_max) {
  n = (n + 3) / 4 * 4;
  return (int)std::max<long long>(1, std::min<long long>(n, si_max));
}

static slh_status create_solver(const slh_problem* problem, void* hip_stream, slh_alloc_fn alloc,
                                slh_free_fn free_fn, void* ctx, bool static_mem,
                                slh_solver** out) {
  if (!out) return fail(SLH_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  slh_status v = validate(problem, true);
  if (v != SLH_OK) return v;
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(SLH_E_INVALID_ARG, "alloc and free_fn must both be set or both be NULL");
  if (static_mem && sizes_of(problem).bytes > kScratchBytes)
    return fail(SLH_E_REJECTED, "the problem needs " + std::to_string(sizes_of(problem).bytes) +
                                    " bytes of device memory, above the static scratch of " +
                                    std::to_string(kScratchBytes) + " bytes");
  slh_solver* s = new (std::nothrow) slh_solver();
  if (!s) return fail(SLH_E_OUT_OF_MEMORY, "host allocation failed");
  if (static_mem) {
    char* base = nullptr;
    int dev = -1;
    const slh_status r = scratch_acquire(&dev, &base);
    if (r != SLH_OK) {
      delete s;
      return r;
    }
    s->static_mem = true;
    s->static_dev = dev;
    s->bump_base = base;
    s->bump_len = kScratchBytes;
    s->use_graphs = false;  // instantiating a graph may allocate
  }
  s->prob = *problem;
  s->z = sizes_of(problem);
  s->stream = (hipStream_t)hip_stream;
  s->alloc = alloc;
  s->free_fn = free_fn;
  s->ctx = ctx;
  const long long nc = s->z.n_cells;
  s->h_sig_s.assign(problem->sigma_s, problem->sigma_s + nc);
  s->h_sig_a.assign(problem->sigma_a, problem->sigma_a + nc);
  s->h_q.assign(problem->q, problem->q + nc);
  s->n_lim_max = problem->n_s < 0 ? 0x7fffffff : problem->n_s;
  if (problem->n_s_cell) {
    s->h_ns.resize(nc);
    s->n_lim_max = 0;
    for (long long i = 0; i < nc; ++i) {
      s->h_ns[i] = problem->n_s_cell[i] < 0 ? 0x7fffffff : problem->n_s_cell[i];
      s->n_lim_max = std::max(s->n_lim_max, s->h_ns[i]);
    }
  }
  s->horizon = problem->steady ? horizon_of(problem) : 0.0;
  // steady pure MC (no limit in any cell): the remap is unnecessary (Sec. 3)
  bool all_unlimited = problem->n_s < 0;
  if (problem->n_s_cell) {
    all_unlimited = true;
    for (long long i = 0; i < nc; ++i) all_unlimited = all_unlimited && problem->n_s_cell[i] < 0;
  }
  s->skip_remap = problem->steady && all_unlimited;
  s->prob.sigma_s = s->prob.sigma_a = s->prob.q = nullptr;
  s->prob.n_s_cell = nullptr;
  if (problem->inflow) s->h_inflow.assign(problem->inflow, problem->inflow + s->z.n_faces);
  s->prob.inflow = nullptr;
  s->hx = (problem->x_hi - problem->x_lo) / problem->nx;
  s->hy = (problem->y_hi - problem->y_lo) / problem->ny;
  s->area = s->hx * s->hy;
  // steady state: weights and fluxes per unit time
  s->adt = problem->steady ? s->area : s->area * problem->dt;
  s->tau = problem->time_closure > 0.0 ? problem->time_closure : 2.0;
  s->si_tol = problem->si_tol > 0.0 ? problem->si_tol : 1e-12;
  s->si_max = problem->si_max_iter > 0 ? problem->si_max_iter : 200;
  s->thin_margin = (long long)ceil(4.0 * sqrt((double)s->z.cap)) + 16;
  // first batch of source iterations per step: for the plain iteration the
  // count at which the largest scattering ratio c = sigma_s / sigma_e, its
  // worst-case contraction, reaches the tolerance; 16 with the diffusion
  // correction (and 16 CG steps per correction), 64 conjugate-gradient steps
  // for the diffusion closing stage (the batches adapt once the first steps
  // are settled; a batch too short costs a rerun of the step, one too long
  // only launches that return at once)
  if (s->z.diffusion) {
    s->si_batch = round_batch(64, s->si_max);
  } else if (s->z.dsa) {
    s->si_batch = round_batch(16, s->si_max);
  } else {
    double c = 0.0;
    const double tt = time_term(problem);
    for (long long i = 0; i < s->z.n_cells; ++i) {
      const double se = s->h_sig_a[i] + s->h_sig_s[i] + tt;
      if (se > 0.0) c = std::max(c, s->h_sig_s[i] / se);
    }
    const double n = c <= 0.0 ? 1.0 : c >= 1.0 ? 64.0 : ceil(log(s->si_tol) / log(c)) + 2.0;
    s->si_batch = round_batch((long long)std::min(64.0, std::max(8.0, n)), s->si_max);
  }
  slh_status r = setup(s);
  if (r != SLH_OK) {
    s->release();
    if (s->static_mem) scratch_release(s->static_dev);
    delete s;
    return r;
  }
  {
    static std::mutex mu;  // the occupancy query is cached per process
    std::lock_guard<std::mutex> lk(mu);
    s->grid1 = mc_pass_grid(s->z.fp32, 1, s->z.cap + s->z.n_src_cap);
    s->grid2 = mc_pass_grid(s->z.fp32, 2, s->z.cap + s->z.n_src_cap);
  }
  *out = s;
  return SLH_OK;
}

extern "C" slh_status slh_create(const slh_problem* problem, void* hip_stream,
                                 slh_alloc_fn alloc, slh_free_fn free_fn, void* ctx,
                                 slh_solver** out) {
  return create_solver(problem, hip_stream, alloc, free_fn, ctx, false, out);
}

extern "C" slh_status slh_create_static(const slh_problem* problem, void* hip_stream,
                                        slh_solver** out) {
  return create_solver(problem, hip_stream, nullptr, nullptr, nullptr, true, out);
}

extern "C" slh_status slh_advance(slh_solver* s, int32_t n_steps) {
  if (!s) return fail(SLH_E_INVALID_ARG, "solver is NULL");
  if (n_steps < 1) return fail(SLH_E_INVALID_ARG, "n_steps must be >= 1");
  for (int k = 0; k < n_steps; ++k) {
    const slh_status r = run_step(s, s->si_batch);
    if (r != SLH_OK) return r;
  }
  return SLH_OK;
}

// Batch for running a halted step again: the iterations it did plus an
// estimate of those it still needs from the contraction of its last two
// iterate changes, rho = |d_k| / |d_{k-1}|, as log(tol |phi| / |d_k|) / log rho,
// with a quarter more and four to spare; the limit si_max when there is no
// estimate (fewer than two iterations, no contraction).
static int restart_batch(const DevState& d, double tol, int si_max) {
  const double dn = sqrt(d.si.dn2), dp = sqrt(d.si.dn2_prev), nrm = sqrt(d.si.nrm2);
  if (d.si.iter < 2 || !(dn > 0.0) || !(dp > 0.0) || !(nrm > 0.0) || !isfinite(dn) ||
      !isfinite(dp) || !isfinite(nrm))
    return si_max;
  const double rho = dn / dp, target = tol * nrm;
  if (!(rho < 0.99)) return si_max;
  if (dn <= target) return round_batch((long long)d.si.iter + 4, si_max);
  const double more = log(target / dn) / log(rho);
  if (!(more < (double)si_max)) return si_max;
  return round_batch((long long)d.si.iter + (long long)ceil(1.25 * more) + 4, si_max);
}

// Waits for the enqueued steps and runs again those that a halted batch left
// undone.  A halted step and every step after it returned from each kernel at
// once, so the device holds the state at the start of the halted step: it is
// run with the batch restart_batch estimates (the full limit si_max if the
// same step halts a second time), the ones after it with a doubled batch (at
// least the estimate), and the check repeats until no step halted.  The batch
// then follows the last step's iteration count (an eighth more, plus two, in
// multiples of four).
static slh_status settle(slh_solver* s, DevState* out = nullptr) {
  DevState d;
  for (;;) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    COPY_SYNC(&d, s->st, sizeof(DevState), hipMemcpyDeviceToHost);
    if (!d.halt) break;
    const long long lost = s->step - (long long)d.step;
    if (lost < 1) return fail(SLH_E_STATE, "a halted step that was not enqueued");
    if (s->timing) s->ev_used -= std::min<size_t>(s->ev_used, (size_t)lost);
    s->cur ^= (int)(lost & 1);
    s->step -= lost;
    s->restarts += (unsigned long long)lost;
    const int rb = d.step == s->last_halted ? s->si_max : restart_batch(d, s->si_tol, s->si_max);
    s->last_halted = d.step;
    s->si_batch = std::max(round_batch(2ll * s->si_batch, s->si_max), rb < s->si_max ? rb : 0);
    s->cg_batch = kDsaMaxIter;  // the halt may have come from a correction
    HIP_TRY(hipMemsetAsync(&s->st->halt, 0, sizeof(int), s->stream));
    slh_status r = run_step(s, rb);
    for (long long k = 1; k < lost && r == SLH_OK; ++k) r = run_step(s, s->si_batch);
    if (r != SLH_OK) return r;
  }
  if (s->unsettled && !s->skip_remap && d.si.iter > 0) {
    s->si_batch = round_batch(d.si.iter + d.si.iter / 8 + 2, s->si_max);
    if (d.dsa_iter_max > 0)  // a quarter more than the step's longest correction, plus two
      s->cg_batch = std::min(kDsaMaxIter, round_batch(d.dsa_iter_max + d.dsa_iter_max / 4 + 2,
                                                      kDsaMaxIter));
  }
  s->unsettled = false;
  if (out) *out = d;
  return SLH_OK;
}

extern "C" slh_status slh_set_si_batch(slh_solver* s, int32_t n) {
  if (!s) return fail(SLH_E_INVALID_ARG, "solver is NULL");
  if (n < 1) return fail(SLH_E_INVALID_ARG, "the batch must be >= 1");
  s->si_batch = n < s->si_max ? n : s->si_max;
  s->cg_batch = n < kDsaMaxIter ? n : kDsaMaxIter;
  return SLH_OK;
}

extern "C" slh_status slh_set_graphs(slh_solver* s, int32_t enable) {
  if (!s) return fail(SLH_E_INVALID_ARG, "solver is NULL");
  if (s->static_mem && enable)
    return fail(SLH_E_STATE, "a static solver launches its kernels directly (no graphs)");
  s->use_graphs = enable != 0;
  return SLH_OK;
}

extern "C" slh_status slh_set_timing(slh_solver* s, int32_t enable) {
  if (!s) return fail(SLH_E_INVALID_ARG, "solver is NULL");
  if (s->static_mem && enable) return fail(SLH_E_STATE, "a static solver records no events");
  s->timing = enable != 0;
  return SLH_OK;
}

// Reads the device state once every enqueued step is done.
static slh_status read_state(slh_solver* s, DevState* d) {
  const slh_status r = settle(s, d);
  if (r != SLH_OK) return r;
  return collect_events(s);
}

extern "C" slh_status slh_synchronize(slh_solver* s) {
  if (!s) return fail(SLH_E_INVALID_ARG, "solver is NULL");
  DevState d;
  const slh_status r = read_state(s, &d);
  if (r != SLH_OK) return r;
  const int f = d.acc_numeric & ~s->rep_numeric;
  const unsigned long long unconv = d.acc_unconv - s->rep_unconv;
  s->rep_numeric = d.acc_numeric;
  s->rep_unconv = d.acc_unconv;
  if (f)
    return fail(SLH_E_NUMERIC,
                std::string("numeric fault in a step since the last synchronisation: ") +
                    ((f & 1) ? "a cell majorant or their sum is not finite; " : "") +
                    ((f & 2) ? "a history ended with a non-finite weight or tally; " : "") +
                    ((f & 4) ? "the emission exceeded the source bank; " : "") +
                    ((f & 8) ? "the source-iteration residual is not finite; " : "") +
                    ((f & 16) ? "histories reached the 2^26-segment guard" : ""));
  if (unconv)
    return fail(SLH_E_NOT_CONVERGED, std::to_string(unconv) +
                                         " step(s) since the last synchronisation stopped the "
                                         "source iteration at si_max_iter");
  return SLH_OK;
}

static const double* flux_ptr(slh_solver* s, int32_t which, long long* n) {
  const long long nc = s->z.n_cells;
  *n = nc;
  switch (which) {
    case SLH_FLUX_REMAP: return s->phi_R;
    case SLH_FLUX_PRE: return s->phi_pre;
    case SLH_FLUX_POST: return s->phi_post;
    case SLH_FLUX_COLLIDED_NODAL: *n = 4 * nc; return s->phi_c;
    default: return nullptr;
  }
}

extern "C" slh_status slh_get_flux(slh_solver* s, int32_t which, double* host_out) {
  if (!s || !host_out) return fail(SLH_E_INVALID_ARG, "NULL argument");
  long long n;
  const double* p = flux_ptr(s, which, &n);
  if (!p) return fail(SLH_E_INVALID_ARG, "unknown flux kind");
  const slh_status r = settle(s);
  if (r != SLH_OK) return r;
  HIP_TRY(hipMemcpyAsync(host_out, p, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return SLH_OK;
}

extern "C" slh_status slh_get_flux_device(slh_solver* s, int32_t which, double* dev_out) {
  if (!s || !dev_out) return fail(SLH_E_INVALID_ARG, "NULL argument");
  long long n;
  const double* p = flux_ptr(s, which, &n);
  if (!p) return fail(SLH_E_INVALID_ARG, "unknown flux kind");
  // a step that halted must run again before its flux can be taken: wait
  // for the steps enqueued since the last settle, if any
  const slh_status r = settle(s);
  if (r != SLH_OK) return r;
  HIP_TRY(hipMemcpyAsync(dev_out, p, sizeof(double) * n, hipMemcpyDeviceToDevice, s->stream));
  return SLH_OK;
}

extern "C" slh_status slh_get_balance(slh_solver* s, int32_t pass, slh_balance* out) {
  if (!s || !out) return fail(SLH_E_INVALID_ARG, "NULL argument");
  if (pass != 1 && pass != 2) return fail(SLH_E_INVALID_ARG, "pass must be 1 or 2");
  {
    const slh_status r = settle(s);
    if (r != SLH_OK) return r;
  }
  BalStore b;
  HIP_TRY(hipMemcpyAsync(&b, s->bal_store + (pass - 1), sizeof(BalStore), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  double v[B_NFIELDS];
  for (int f = 0; f < B_NFIELDS; ++f)
    v[f] = fix_value((long long)b.bal[2 * f], (long long)b.bal[2 * f + 1], b.unit_W);
  out->emitted = v[B_EMITTED];
  out->absorbed = v[B_ABSORBED];
  out->scattered = v[B_SCATTERED];
  out->leaked = v[B_LEAKED];
  out->census = v[B_CENSUS];
  out->cutoff = v[B_CUTOFF];
  out->source_w = v[B_SOURCE_W];
  out->census_in_w = v[B_CENSUS_IN_W];
  out->segments = b.segments;
  out->particles = b.particles;
  out->majorant_sum = b.sumM;
  out->weight_quantum = b.wq;
  out->source_particles = (uint64_t)b.n_emit;
  out->killed = b.killed;
  return SLH_OK;
}

extern "C" slh_status slh_get_stats(slh_solver* s, slh_stats* out) {
  if (!s || !out) return fail(SLH_E_INVALID_ARG, "NULL argument");
  DevState d;
  const slh_status r = read_state(s, &d);
  if (r != SLH_OK) return r;
  BalStore b[2];
  COPY_SYNC(b, s->bal_store, sizeof(b), hipMemcpyDeviceToHost);
  memset(out, 0, sizeof(*out));
  out->step = s->step;
  out->si_iterations = d.si.iter;
  const double dn = sqrt(d.si.dn2), nrm = sqrt(d.si.nrm2);
  out->si_residual = nrm > 0.0 ? dn / nrm : 0.0;
  out->si_converged = d.si.conv ? 1 : 0;
  out->census_alive = (int64_t)b[1].alive;
  out->census_kept = d.n_kept;
  out->thin_factor = d.thin_factor;
  out->segments_total = b[0].segments + b[1].segments;
  out->ms_kernel_mc_total = s->k_ms[0];
  out->ms_kernel_remap_total = s->k_ms[1];
  out->seg_mc_total = d.acc_seg[0];
  out->seg_remap_total = d.acc_seg[1];
  out->census_in_total = d.acc_census_in;
  out->census_out_total = d.acc_census_out;
  out->steps_total = d.acc_steps;
  out->thin_overflow_total = d.acc_thin_overflow;
  out->graph_launches_total = s->graph_launches;
  out->host_waits_total = 0;  // slh_advance never waits
  out->killed_total = d.acc_killed;
  out->dsa_corrections = d.dsa_corrections;
  out->dsa_iterations = d.dsa_iter_total;
  out->dsa_unconverged = d.dsa_unconv;
  out->si_unconverged_total = d.acc_unconv;
  out->si_batch = s->skip_remap ? 0 : s->si_batch;
  out->si_restarts_total = s->restarts;
  out->numeric_flags = d.acc_numeric;
  if (s->have_stage) {
    out->ms_mc = s->stage_ms[0];
    out->ms_dg = s->stage_ms[1];
    out->ms_remap = s->stage_ms[2];
    out->ms_census = s->stage_ms[3];
  }
  return SLH_OK;
}

// The first cnt census records of the current bank, as host fields in the
// solver's precision (px, py: cell-local).
template <typename R>
static slh_status read_bank(slh_solver* s, long long cnt, std::vector<R>* f5,
                            std::vector<int32_t>& cell, std::vector<uint64_t>& hid) {
  std::vector<StageRec<R>> recs(cnt);
  COPY_SYNC(recs.data(), s->bank_mem[s->cur], sizeof(StageRec<R>) * cnt, hipMemcpyDeviceToHost);
  for (int k = 0; k < 5; ++k) f5[k].resize(cnt);
  cell.resize(cnt);
  hid.resize(cnt);
  for (long long i = 0; i < cnt; ++i) {
    const StageRec<R>& r = recs[i];
    f5[0][i] = r.px; f5[1][i] = r.py; f5[2][i] = r.ox; f5[3][i] = r.oy; f5[4][i] = r.w;
    cell[i] = r.cell;
    hid[i] = r.hid;
  }
  return SLH_OK;
}

// Writes cnt census records into the current bank from SoA host arrays.
template <typename R>
static slh_status write_bank(slh_solver* s, long long cnt, const R* const* f5,
                             const int32_t* cell, const uint64_t* hid) {
  std::vector<StageRec<R>> recs(cnt);
  for (long long i = 0; i < cnt; ++i) {
    StageRec<R>& r = recs[i];
    memset(&r, 0, sizeof(r));
    r.px = f5[0][i]; r.py = f5[1][i]; r.ox = f5[2][i]; r.oy = f5[3][i]; r.w = f5[4][i];
    r.cell = cell[i];
    r.hid = hid[i];
  }
  if (cnt) COPY_SYNC(s->bank_mem[s->cur], recs.data(), sizeof(StageRec<R>) * cnt,
                     hipMemcpyHostToDevice);
  return SLH_OK;
}

extern "C" slh_status slh_get_census(slh_solver* s, int64_t* n, double* x, double* y,
                                     double* ox, double* oy, double* w, int32_t* cell,
                                     uint64_t* hid) {
  if (!s || !n) return fail(SLH_E_INVALID_ARG, "NULL argument");
  DevState d;
  {
    const slh_status r = settle(s, &d);
    if (r != SLH_OK) return r;
  }
  const long long cnt = d.n_in;
  *n = cnt;
  if (cnt == 0) return SLH_OK;
  const slh_problem& p = s->prob;
  std::vector<int32_t> c;
  std::vector<uint64_t> h;
  std::vector<double> f[5];
  if (s->z.fp32) {
    std::vector<float> t[5];
    const slh_status r = read_bank<float>(s, cnt, t, c, h);
    if (r != SLH_OK) return r;
    for (int k = 0; k < 5; ++k) f[k].assign(t[k].begin(), t[k].end());
  } else {
    const slh_status r = read_bank<double>(s, cnt, f, c, h);
    if (r != SLH_OK) return r;
  }
  for (long long i = 0; i < cnt; ++i) {
    const int ix = c[i] % p.nx, iy = c[i] / p.nx;
    if (x) x[i] = p.x_lo + s->hx * ix + f[0][i];
    if (y) y[i] = p.y_lo + s->hy * iy + f[1][i];
    if (ox) ox[i] = f[2][i];
    if (oy) oy[i] = f[3][i];
    if (w) w[i] = f[4][i];
    if (cell) cell[i] = c[i];
    if (hid) hid[i] = h[i];
  }
  return SLH_OK;
}

// Checkpoint layout: ten 8-byte header words (magic, abi, step, precision,
// count, maxabs, nx, ny, seed, cap), then the raw bank arrays (px, py, ox, oy,
// w in the solver's precision, hid, cell).
static const uint64_t kMagic = 0x534c48434b505432ull;  // "SLHCKPT2"
static const size_t kCkptHead = 10 * 8;

extern "C" slh_status slh_save(slh_solver* s, void* buf, size_t* len) {
  if (!s || !len) return fail(SLH_E_INVALID_ARG, "NULL argument");
  DevState d;
  {
    const slh_status r = settle(s, &d);
    if (r != SLH_OK) return r;
  }
  const long long cnt = d.n_in;
  const size_t need = kCkptHead + (size_t)cnt * ((s->z.fp32 ? 4 : 8) * 5 + 8 + 4);
  if (!buf) { *len = need; return SLH_OK; }
  if (*len < need) return fail(SLH_E_INVALID_ARG, "buffer too small");
  uint64_t* h = (uint64_t*)buf;
  h[0] = kMagic;
  h[1] = SLH_ABI_VERSION;
  h[2] = (uint64_t)s->step;
  h[3] = (uint64_t)s->z.fp32;
  h[4] = (uint64_t)cnt;
  memcpy(&h[5], &d.maxabs_w, 8);
  h[6] = (uint64_t)s->prob.nx;
  h[7] = (uint64_t)s->prob.ny;
  h[8] = s->prob.seed;
  h[9] = (uint64_t)s->z.cap;
  char* out = (char*)buf + kCkptHead;
  if (cnt > 0) {
    std::vector<int32_t> c;
    std::vector<uint64_t> hh;
    const size_t rb = s->z.fp32 ? 4 : 8;
    if (s->z.fp32) {
      std::vector<float> f[5];
      const slh_status r = read_bank<float>(s, cnt, f, c, hh);
      if (r != SLH_OK) return r;
      for (int k = 0; k < 5; ++k, out += rb * cnt) memcpy(out, f[k].data(), rb * cnt);
    } else {
      std::vector<double> f[5];
      const slh_status r = read_bank<double>(s, cnt, f, c, hh);
      if (r != SLH_OK) return r;
      for (int k = 0; k < 5; ++k, out += rb * cnt) memcpy(out, f[k].data(), rb * cnt);
    }
    memcpy(out, hh.data(), 8 * cnt);
    out += 8 * cnt;
    memcpy(out, c.data(), 4 * cnt);
  }
  *len = need;
  return SLH_OK;
}

// Host-side check of a checkpoint's particles before they reach the device:
// every cell on the mesh, positions inside their cell, directions and
// weights finite, and the stored max |w| (the next pass's fixed-point bound)
// not below any weight.
template <typename R>
static bool ckpt_bank_ok(const char* in, long long cnt, long long n_cells, double hx, double hy,
                         double maxabs) {
  const R* px = (const R*)in;
  const R* py = px + cnt;
  const R* ox = py + cnt;
  const R* oy = ox + cnt;
  const R* w = oy + cnt;
  const int32_t* cell = (const int32_t*)((const char*)(w + cnt) + 8 * cnt);
  if (!(maxabs >= 0.0) || !isfinite(maxabs)) return false;
  for (long long i = 0; i < cnt; ++i) {
    if (cell[i] < 0 || (long long)cell[i] >= n_cells) return false;
    if (i > 0 && cell[i] < cell[i - 1]) return false;  // banks are ordered by cell
    const double x = px[i], y = py[i], a = ox[i], b = oy[i], v = w[i];
    // (with a relative slack of 1e-6 for the rounding of FP32 banks)
    if (!(x >= 0.0 && x <= hx * (1.0 + 1e-6) && y >= 0.0 && y <= hy * (1.0 + 1e-6))) return false;
    if (!(fabs(a) <= 1.0 + 1e-6 && fabs(b) <= 1.0 + 1e-6) || !isfinite(v) || fabs(v) > maxabs)
      return false;
  }
  return true;
}

extern "C" slh_status slh_load(slh_solver* s, const void* buf, size_t len) {
  if (!s || !buf) return fail(SLH_E_INVALID_ARG, "NULL argument");
  if (len < kCkptHead) return fail(SLH_E_INVALID_ARG, "checkpoint truncated");
  const uint64_t* h = (const uint64_t*)buf;
  if (h[0] != kMagic || h[1] != SLH_ABI_VERSION) return fail(SLH_E_INVALID_ARG, "not a checkpoint");
  if (h[3] != (uint64_t)s->z.fp32) return fail(SLH_E_INVALID_ARG, "checkpoint precision differs");
  if (h[6] != (uint64_t)s->prob.nx || h[7] != (uint64_t)s->prob.ny)
    return fail(SLH_E_INVALID_ARG, "checkpoint is of another mesh");
  if (h[8] != s->prob.seed) return fail(SLH_E_INVALID_ARG, "checkpoint has another seed");
  const long long cnt = (long long)h[4];
  if (cnt < 0 || cnt > s->z.cap) return fail(SLH_E_INVALID_ARG, "checkpoint bank exceeds the cap");
  const size_t rb = s->z.fp32 ? 4 : 8;
  if (len < kCkptHead + (size_t)cnt * (rb * 5 + 8 + 4))
    return fail(SLH_E_INVALID_ARG, "checkpoint truncated");
  double maxabs;
  memcpy(&maxabs, &h[5], 8);
  const char* in = (const char*)buf + kCkptHead;
  const bool ok = s->z.fp32 ? ckpt_bank_ok<float>(in, cnt, s->z.n_cells, s->hx, s->hy, maxabs)
                            : ckpt_bank_ok<double>(in, cnt, s->z.n_cells, s->hx, s->hy, maxabs);
  if (!ok) return fail(SLH_E_INVALID_ARG, "checkpoint particles are not valid for this problem");
  {
    const slh_status r = settle(s);  // steps still enqueued finish first
    if (r != SLH_OK) return r;
  }
  {
    const uint64_t* hh = (const uint64_t*)(in + rb * 5 * cnt);
    const int32_t* cc = (const int32_t*)(in + rb * 5 * cnt + 8 * cnt);
    slh_status r;
    if (s->z.fp32) {
      const float* f[5];
      for (int k = 0; k < 5; ++k) f[k] = (const float*)(in + rb * k * cnt);
      r = write_bank<float>(s, cnt, f, cc, hh);
    } else {
      const double* f[5];
      for (int k = 0; k < 5; ++k) f[k] = (const double*)(in + rb * k * cnt);
      r = write_bank<double>(s, cnt, f, cc, hh);
    }
    if (r != SLH_OK) return r;
  }
  hipLaunchKernelGGL(k_state_set_bank, dim3(1), dim3(1), 0, s->stream, s->st, cnt, maxabs,
                     (unsigned long long)h[2]);
  HIP_TRY(hipGetLastError());
  // the loaded bank's cohort ranks
  if (s->z.fp32)
    HIP_TRY(launch_bank_cells<float>((const StageRec<float>*)s->bank_mem[s->cur], cnt,
                                     s->skey[0], s->stream));
  else
    HIP_TRY(launch_bank_cells<double>((const StageRec<double>*)s->bank_mem[s->cur], cnt,
                                      s->skey[0], s->stream));
  HIP_TRY(launch_cohort_ranks(s->skey[0], &s->st->n_in, cnt, s->cstart, s->crank[s->cur], s->st,
                              s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->step = (long long)h[2];
  {
    const slh_status r = collect_events(s);
    if (r != SLH_OK) return r;
  }
  s->k_ms[0] = s->k_ms[1] = 0.0;
  s->have_stage = false;
  s->rep_unconv = 0ull;
  s->rep_numeric = 0;
  return SLH_OK;
}

extern "C" void slh_destroy(slh_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  s->release();
  if (s->static_mem) scratch_release(s->static_dev);
  delete s;
}

extern "C" slh_status slh_qmc_points(uint64_t seed, uint64_t step, uint32_t pass,
                                     uint32_t population, uint64_t cohort, uint32_t dim0,
                                     uint32_t n_dims, uint32_t index0, uint32_t n, int32_t points,
                                     uint32_t* dev_out, void* hip_stream) {
  if (!dev_out && n && n_dims) return fail(SLH_E_INVALID_ARG, "dev_out is NULL");
  if (points != SLH_SOBOL_OWEN && points != SLH_PRNG && points != SLH_HALTON)
    return fail(SLH_E_INVALID_ARG, "unknown point set");
  if ((uint64_t)index0 + n > 0x100000000ull) return fail(SLH_E_INVALID_ARG, "index range > 2^32");
  static uint32_t* table = nullptr;  // per process, device 0 context
  if (!table) {
    uint32_t* t = nullptr;
    HIP_TRY(hipMalloc(&t, 4 * 32 * 32));
    HIP_TRY(hipMemcpy(t, sobol_table_host(), 4 * 32 * 32, hipMemcpyHostToDevice));
    table = t;
  }
  const uint64_t stream = stream_seed(seed, step, pass, population, cohort);
  HIP_TRY(launch_qmc_points(stream, dim0, n_dims, index0, n, points, table, dev_out,
                            (hipStream_t)hip_stream));
  return SLH_OK;
}
