// Collided solve of the hybrid step (step 2 of Sec. 2.2): discrete ordinates
// with bilinear discontinuous Galerkin in space, upwind faces, vacuum inflow,
// and a step-averaged time closure sigma_e = sigma_t + tau/(c dt).  One
// transport sweep per direction and source-iteration sweep.
//
// Element matrices on a cell of size hx x hy, node k = kx + 2 ky at
// (x_kx, y_ky), 1-D factors  M = h/6 [[2,1],[1,2]] (mass) and
// K = 1/2 [[-1,1],[-1,1]] (K[i][j] = int L_i L_j'):
//   A = a Kx(x)My + b Mx(x)Ky + sig_e Mx(x)My
//     + |a| (e_f e_f^T)(x)My + |b| Mx(x)(e_g e_g^T)
// where f (g) is the local index of the x (y) inflow face; the right side is
// (Mx(x)My) S + F up with F up = |a| e_f (x) My up_x + |b| Mx up_y (x) e_g for
// the upwind traces up = (up_x0, up_x1, up_y0, up_y1) (zero on the domain
// boundary).  On the uniform mesh A0 = A - sig_e Mx(x)My and F depend on the
// direction only.
//
// Device layout: one workgroup per direction walks the cells in diagonal
// wavefronts of the direction's upwind order, in chunks of CW cells (a
// diagonal, or a piece of a long one).  Cells of one diagonal have distinct
// rows and columns, so the outflow traces they hand to the next diagonal live
// in two small LDS arrays (one trace per row for the x faces, one per column
// for the y faces).  The workgroup has CW/64 sweeping waves and CW/(64 Q)
// loader waves (Q cells per loader lane).  The loaders keep several chunks of
// nodal sources and material keys in flight in registers and hand each chunk
// over through a two-slot LDS buffer, so the sweeping waves never wait on
// global memory: their only global accesses are the stores of psi_m (a
// wave that mixed loads and stores would have to drain all of them before
// using a loaded value).  After each barrier a sweeping lane turns the upwind
// traces into its cell's solution with the element data prepared before the
// barrier:
//   table mode: psi = B S + G up with B = A^-1 Mx(x)My, G = A^-1 F taken from
//     a per-(direction, material) table staged in LDS (few distinct sigma_e);
//     the loader hands over B S instead of S;
//   cell mode: A is LU-factorised before the barrier and solved after it.
// The solution goes to a per-direction plane, and a second kernel sums
// w_m psi_m over the directions in a fixed order, so the scalar flux does not
// depend on scheduling.  The sources, sigma_e and the planes are stored in the
// sweep's own layouts (anti-diagonals or diagonals, DgArgs), where the cells
// of a chunk are contiguous: a diagonal of a row-major array would touch a
// different cache line in every lane.
#include "slh_common.hpp"

namespace slh {

// 1/a from the hardware reciprocal estimate refined by two Newton steps
// (quadratic convergence from ~2^-26 to full FP64 precision).
__device__ __forceinline__ double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(fma(-a, r, 1.0), r, r);
  r = fma(fma(-a, r, 1.0), r, r);
  return r;
}

// Start of a step's source iteration: phi_c = 0, the iteration state reset
// (block 0), the nodal source of the first iterate
// S = sigma_s/(4 pi) (phi_c + phi_post) with phi_c = 0 (later iterates get
// theirs from the flux reduction), and with reflective sides the buffer of
// reflected traces that the first sweep reads set to zero.
__global__ void k_si_start(int nx, int ny, const double* __restrict__ sig_s,
                           const double* __restrict__ phi_post, double* __restrict__ phi_c,
                           double* __restrict__ S, double* __restrict__ bnd0, long long n_bnd,
                           DevState* st, int si_max) {
  if (st->halt) return;
  const long long n = (long long)nx * ny;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->si.iter = 0;
    st->si.conv = si_max == 0 ? 1 : 0;
    st->si.done = si_max == 0 ? 1 : 0;
    st->si.bad = 0;
    st->si.dn2 = 0.0;
    st->si.dn2_prev = 0.0;
    st->si.nrm2 = 0.0;
    st->dsa_unconv = 0;
    st->dsa_corrections = 0;
    st->dsa_iter_total = 0;
    st->dsa_iter_max = 0;
  }
  const double inv4pi = 0.25 / M_PI;
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long str = (long long)gridDim.x * blockDim.x;
  for (long long i = i0; i < n; i += str) {
    const double ssc = sig_s[i] * inv4pi;
    const double v = ssc * (0.0 + phi_post[i]);
    const int ci = (int)(i % nx), cj = (int)(i / nx);
    reinterpret_cast<double4*>(phi_c)[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    reinterpret_cast<double4*>(S)[lay_pos(nx, ny, ci, cj, true)] = make_double4(v, v, v, v);
    reinterpret_cast<double4*>(S)[n + lay_pos(nx, ny, ci, cj, false)] = make_double4(v, v, v, v);
  }
  for (long long k = i0; k < n_bnd; k += str) bnd0[k] = 0.0;
}

// Direction part of the element: A0 and F (row-major 4x4 each) and the mass
// matrix MM = Mx(x)My.
__device__ void element(double a, double b, double hx, double hy, double A0[4][4],
                        double F[4][4], double MM[4][4]) {
  const int fx = a > 0.0 ? 0 : 1, fy = b > 0.0 ? 0 : 1;
  const double aa = fabs(a), ab = fabs(b);
  const double Mx[2][2] = {{hx / 3.0, hx / 6.0}, {hx / 6.0, hx / 3.0}};
  const double My[2][2] = {{hy / 3.0, hy / 6.0}, {hy / 6.0, hy / 3.0}};
  const double K[2][2] = {{-0.5, 0.5}, {-0.5, 0.5}};
  for (int r = 0; r < 4; ++r) {
    const int kx = r & 1, ky = r >> 1;
    for (int l = 0; l < 4; ++l) {
      const int lx = l & 1, ly = l >> 1;
      double v = a * K[kx][lx] * My[ky][ly] + b * Mx[kx][lx] * K[ky][ly];
      if (kx == fx && lx == fx) v += aa * My[ky][ly];
      if (ky == fy && ly == fy) v += ab * Mx[kx][lx];
      A0[r][l] = v;
      MM[r][l] = Mx[kx][lx] * My[ky][ly];
    }
    F[r][0] = kx == fx ? aa * My[ky][0] : 0.0;
    F[r][1] = kx == fx ? aa * My[ky][1] : 0.0;
    F[r][2] = ky == fy ? ab * Mx[kx][0] : 0.0;
    F[r][3] = ky == fy ? ab * Mx[kx][1] : 0.0;
  }
}

// Per-direction element data [m][32]: A0 then F.
__global__ void k_dg_dirmat(int n_dir, const double* __restrict__ dir, double hx, double hy,
                            double* __restrict__ dm) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_dir) return;
  double A0[4][4], F[4][4], MM[4][4];
  element(dir[3 * m], dir[3 * m + 1], hx, hy, A0, F, MM);
  for (int r = 0; r < 4; ++r)
    for (int l = 0; l < 4; ++l) {
      dm[32 * m + 4 * r + l] = A0[r][l];
      dm[32 * m + 16 + 4 * r + l] = F[r][l];
    }
}

// Table [m][material][32]: B = A^-1 MM then G = A^-1 F (row-major), by
// Gauss-Jordan elimination of [A | MM | F]; the pivots do not vanish (the
// symmetric part of the upwind element matrix is positive definite: mass and
// inflow terms are SPD and the streaming term's symmetric part, the outflow
// minus inflow face mass, becomes |Omega.n| face mass with the inflow term).
__global__ void k_dg_coef(int n_dir, int n_mat, const double* __restrict__ dir,
                          const double* __restrict__ sig_e_mat, double hx, double hy,
                          double* __restrict__ coef) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n_dir * n_mat) return;
  const int m = (int)(t / n_mat), k = (int)(t % n_mat);
  const double se = sig_e_mat[k];
  double A[4][4], F[4][4], MM[4][4], R[4][8];
  element(dir[3 * m], dir[3 * m + 1], hx, hy, A, F, MM);
  for (int r = 0; r < 4; ++r)
    for (int l = 0; l < 4; ++l) {
      A[r][l] += se * MM[r][l];
      R[r][l] = MM[r][l];
      R[r][4 + l] = F[r][l];
    }
  for (int c = 0; c < 4; ++c) {
    const double inv = 1.0 / A[c][c];
    for (int l = 0; l < 4; ++l) A[c][l] *= inv;
    for (int j = 0; j < 8; ++j) R[c][j] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const double f = A[r][c];
      for (int l = 0; l < 4; ++l) A[r][l] -= f * A[c][l];
      for (int j = 0; j < 8; ++j) R[r][j] -= f * R[c][j];
    }
  }
  double* o = coef + t * 32;
  for (int r = 0; r < 4; ++r)
    for (int j = 0; j < 4; ++j) {
      o[4 * r + j] = R[r][j];
      o[16 + 4 * r + j] = R[r][4 + j];
    }
}

hipError_t launch_dg_tables(int n_dir, int n_mat, const double* dir, const double* sig_e_mat,
                            double hx, double hy, double* dirmat, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_dg_dirmat, dim3((n_dir + 63) / 64), dim3(64), 0, s, n_dir, dir, hx, hy,
                     dirmat);
  if (n_mat > 0 && coef) {
    const long long n = (long long)n_dir * n_mat;
    hipLaunchKernelGGL(k_dg_coef, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, n_dir,
                       n_mat, dir, sig_e_mat, hx, hy, coef);
  }
  return hipGetLastError();
}

// Chunks of the sweep: sum over diagonals of ceil(length / cw).
long long dg_chunks(int nx, int ny, int cw) {
  long long n = 0;
  for (int d = 0; d < nx + ny - 1; ++d) {
    const int lo = d - (ny - 1) > 0 ? d - (ny - 1) : 0;
    const int hi = d < nx - 1 ? d : nx - 1;
    n += (hi - lo + cw) / cw;
  }
  return n;
}

constexpr int kDgDepth = 4;  // chunks in flight in the loader wave
constexpr int kDgRow = 34;   // LDS stride of a table row (32 values)

// One chunk in a loader lane: Q cells (source, key, position in the chunk
// or -1).
template <int Q>
struct DgStage {
  double Sx[Q], Sy[Q], Sz[Q], Sw[Q];
  double Kd[Q];  // cell mode: sigma_e
  int Ki[Q];     // table mode: material
  int C[Q];
};

// The sweep of one direction, compiled for each quadrant (APOS: Omega_x > 0,
// BPOS: Omega_y > 0), so that the upwind order costs no selects.  A chunk has
// CW cells; a sweeping lane takes Q of them (positions t, t + CW/Q, ...),
// whose independent solves hide each other's latency, and so does a loader
// lane.
template <bool TABLE, int Q, bool REFL, bool APOS, bool BPOS>
__device__ __forceinline__ void sweep_dir(const DgArgs& g) {
  extern __shared__ double smem[];
  const int nx = g.nx, ny = g.ny;
  const int CW = g.cw;            // cells per chunk, a multiple of 64 Q
  const int n_sw = CW / (64 * Q); // sweeping waves; as many loader waves follow them
  const int n_ld = n_sw;
  const int m = blockIdx.x;
  constexpr bool apos = APOS, bpos = BPOS;
  // LDS: slots S [2][CW] as two double2 halves | keys [2][CW] | coef [n_mat][kDgRow] | faces
  // (the source halves and the table rows are laid out so that a wave's
  // accesses fall in distinct banks: 16-byte lane stride, rows offset by
  // four banks)
  double2* slotA = reinterpret_cast<double2*>(smem);  // S.x, S.y
  double2* slotB = slotA + (size_t)2 * CW;             // S.z, S.w
  double* slotK = smem + (size_t)2 * CW * 4;
  double* coefL = slotK + (size_t)2 * CW;
  const size_t n_coef = TABLE ? (size_t)g.n_mat * kDgRow : 0;
  double* xf = coefL + n_coef;  // 16-byte aligned (80 CW + 272 n_mat bytes in), read as double2
  double* yf = xf + 2 * ny;
  const int n_diag = nx + ny - 1;
  // barriers: one per chunk, padded to whole loader rounds (the padding
  // chunks are empty), so the loader's rounds have no conditional steps
  const int n_pad = (g.n_chunks + kDgDepth - 1) / kDgDepth * kDgDepth;
  auto diag_hi = [&](int dd) __attribute__((always_inline)) { return dd < nx - 1 ? dd : nx - 1; };
  auto diag_lo = [&](int dd) __attribute__((always_inline)) { return dd - (ny - 1) > 0 ? dd - (ny - 1) : 0; };
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool loader = wave >= n_sw;
  const int lane = threadIdx.x & 63;
  const int lw = wave - n_sw;  // loader wave index
  // this direction's layout: A (anti-diagonals) when both components have the
  // same sign; the chunk of upwind diagonal dd is run n_diag - 1 - dd of the
  // layout when Omega_x < 0, and cell i sits at run start - lo + i
  constexpr bool anti = APOS == BPOS;
  const long long lay_base = anti ? 0 : (long long)nx * ny;
  auto run_base = [&](int dd) __attribute__((always_inline)) {
    const int r = apos ? dd : n_diag - 1 - dd;
    return lay_run(nx, ny, r) - (long long)diag_lo(r) + lay_base;
  };

  // ---- loader state: ring of kDgDepth chunks, Q cells per lane ----
  DgStage<Q> r0s, r1s, r2s, r3s;
  int fd = 0, fp = 0;   // fetch front: diagonal, first position
  // Every lane issues the same loads in every stage (a position without a
  // cell reads cell 0 and is marked -1): with no branch around the loads the
  // compiler can wait for one stage while the younger ones stay in flight.
  auto fetch = [&](DgStage<Q>& st) __attribute__((always_inline)) {
    const bool live = fd < n_diag;
    const int hi = live ? diag_hi(fd) : -1;
    const int dl = live ? fd : n_diag - 1;  // a real diagonal for the addresses
    const int dlo = diag_lo(dl), dhi = diag_hi(dl);
    const long long rb = run_base(dl);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int tq = lane + 64 * (lw + n_ld * q);
      const int ip = fp + tq;
      const bool ok = ip <= hi;
      // clamp the position onto the diagonal, so that every lane's address
      // is a real cell and no branch guards the loads
      const int ipc = ip < dlo ? dlo : (ip < dhi ? ip : dhi);
      const int i = apos ? ipc : nx - 1 - ipc;
      const long long c = rb + i;  // position in this direction's layout
      st.C[q] = ok ? tq : -1;
      if (TABLE) st.Ki[q] = g.mat_id[c];
      else st.Kd[q] = g.sig_e[c];
      const double4 v = reinterpret_cast<const double4*>(g.src)[c];
      st.Sx[q] = v.x;
      st.Sy[q] = v.y;
      st.Sz[q] = v.z;
      st.Sw[q] = v.w;
    }
    if (live) {
      fp += CW;
      if (fp > hi) {
        ++fd;
        fp = fd < n_diag ? diag_lo(fd) : 0;
      }
    }
  };
  // Table mode hands over B S (B from the staged table) instead of S, which
  // takes a matrix-vector product off the sweeping lanes' critical path.
  auto hand_over = [&](const DgStage<Q>& st, int slot) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (st.C[q] >= 0) {
        double4 v = make_double4(st.Sx[q], st.Sy[q], st.Sz[q], st.Sw[q]);
        if (TABLE) {
          const double* c = coefL + (size_t)st.Ki[q] * kDgRow;
          v = make_double4(c[0] * st.Sx[q] + c[1] * st.Sy[q] + c[2] * st.Sz[q] + c[3] * st.Sw[q],
                           c[4] * st.Sx[q] + c[5] * st.Sy[q] + c[6] * st.Sz[q] + c[7] * st.Sw[q],
                           c[8] * st.Sx[q] + c[9] * st.Sy[q] + c[10] * st.Sz[q] + c[11] * st.Sw[q],
                           c[12] * st.Sx[q] + c[13] * st.Sy[q] + c[14] * st.Sz[q] + c[15] * st.Sw[q]);
        }
        slotA[slot * CW + st.C[q]] = make_double2(v.x, v.y);
        slotB[slot * CW + st.C[q]] = make_double2(v.z, v.w);
        slotK[slot * CW + st.C[q]] = TABLE ? (double)st.Ki[q] : st.Kd[q];
      }
  };
  if (loader) {
    fetch(r0s);
    fetch(r1s);
    fetch(r2s);
    fetch(r3s);
  }
  // upwind faces: zero (vacuum) or, on a reflective side, the previous
  // iteration's outflow of the mirrored direction
  // (REFL: some side reflects and g.bnd holds the traces)
  const size_t sb = (size_t)2 * (nx + ny);  // boundary traces per direction
  const int it = REFL ? g.st->si.iter : 0;
  const bool rx_in = REFL && (g.bc & (apos ? 1 : 2)) != 0;
  const bool ry_in = REFL && (g.bc & (bpos ? 4 : 8)) != 0;
  const bool rx_out = REFL && (g.bc & (apos ? 2 : 1)) != 0;
  const bool ry_out = REFL && (g.bc & (bpos ? 8 : 4)) != 0;
  const double* b_in = REFL ? g.bnd + (size_t)((it + 1) & 1) * g.n_dir * sb : nullptr;
  double* b_out = REFL ? g.bnd + ((size_t)(it & 1) * g.n_dir + m) * sb : nullptr;
  if (rx_in || ry_in) {
    for (int k = threadIdx.x; k < 2 * (nx + ny); k += blockDim.x) {
      double v = 0.0;
      if (k < 2 * ny) {
        if (rx_in) v = b_in[(size_t)g.refl_x[m] * sb + k];
      } else if (ry_in) {
        v = b_in[(size_t)g.refl_y[m] * sb + k];
      }
      xf[k] = v;  // yf = xf + 2 ny
    }
  } else {
    for (int k = threadIdx.x; k < 2 * (nx + ny); k += blockDim.x) xf[k] = 0.0;
  }
  if (TABLE) {
    const double* src = g.coef + (size_t)m * g.n_mat * 32;
    for (int k = threadIdx.x; k < g.n_mat * 32; k += blockDim.x)
      coefL[(k >> 5) * kDgRow + (k & 31)] = src[k];
  }
  __syncthreads();  // faces zeroed, table staged
  if (loader) {
    hand_over(r0s, 0);
    fetch(r0s);
  }
  __syncthreads();  // chunk 0 in slot 0

  if (loader) {
    // before barrier k, chunk k + 1 goes to slot (k + 1) & 1; it sits in
    // ring entry (k + 1) % depth, loaded depth - 1 rounds earlier
    for (int k0 = 0; k0 < n_pad; k0 += kDgDepth) {
#define SLH_DG_LOAD_STEP(U, R)    \
  hand_over(R, (k0 + U + 1) & 1); \
  fetch(R);                       \
  __syncthreads();
      SLH_DG_LOAD_STEP(0, r1s)
      SLH_DG_LOAD_STEP(1, r2s)
      SLH_DG_LOAD_STEP(2, r3s)
      SLH_DG_LOAD_STEP(3, r0s)
#undef SLH_DG_LOAD_STEP
    }
    return;
  }

  // ---- sweeping lanes: Q cells each ----
  const int t = threadIdx.x;
  const int span = CW / Q;  // chunk positions t + r span, r < Q
  double dmA[16], dmF[16];  // cell mode: direction element data
  if (!TABLE) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      dmA[k] = g.dirmat[32 * m + k];
      dmF[k] = g.dirmat[32 * m + 16 + k];
    }
  }
  const double hx = g.hx, hy = g.hy;
  const double MM[4][4] = {
      {hx * hy / 9.0, hx * hy / 18.0, hx * hy / 18.0, hx * hy / 36.0},
      {hx * hy / 18.0, hx * hy / 9.0, hx * hy / 36.0, hx * hy / 18.0},
      {hx * hy / 18.0, hx * hy / 36.0, hx * hy / 9.0, hx * hy / 18.0},
      {hx * hy / 36.0, hx * hy / 18.0, hx * hy / 18.0, hx * hy / 9.0}};
  double4* __restrict__ out = reinterpret_cast<double4*>(g.psi + (long long)m * 4 * nx * ny);
  int cd = 0, cp = 0;  // next chunk to prepare
  // the prepared cells: present, indices (0 for an absent cell, whose
  // arithmetic runs on stale data and is dropped) and layout position
  bool c_has[Q];
  int c_i[Q], c_j[Q];
  long long c_pos[Q];
  double P[Q][16];    // table: G; cell mode: B^-1, D, S^-1, G of the block factorisation
  double r0[Q][4];    // table: B S; cell mode: MM S
  auto prepare = [&](int slot) __attribute__((always_inline)) {
    const bool live = cd < n_diag;
    const int hi = live ? diag_hi(cd) : -1;
    const long long rb = run_base(live ? cd : n_diag - 1);
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      const int tr = t + r * span;
      const int ip = cp + tr;
      const bool h = ip <= hi;
      const int jp = cd - ip;
      c_has[r] = h;
      c_i[r] = h ? (apos ? ip : nx - 1 - ip) : 0;
      c_j[r] = h ? (bpos ? jp : ny - 1 - jp) : 0;
      c_pos[r] = rb + c_i[r];
      const double2 sa = slotA[slot * CW + tr], sb = slotB[slot * CW + tr];
      const double4 S = make_double4(sa.x, sa.y, sb.x, sb.y);
      const double key = slotK[slot * CW + tr];
      if (TABLE) {
        const double* c = coefL + (size_t)(h ? (int)key : 0) * kDgRow;
        r0[r][0] = S.x;  // B S, formed by the loader
        r0[r][1] = S.y;
        r0[r][2] = S.z;
        r0[r][3] = S.w;
#pragma unroll
        for (int k = 0; k < 16; ++k) P[r][k] = c[16 + k];
      } else {
        double A[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
          for (int l = 0; l < 4; ++l) A[a][l] = dmA[4 * a + l] + key * MM[a][l];
          r0[r][a] = MM[a][0] * S.x + MM[a][1] * S.y + MM[a][2] * S.z + MM[a][3] * S.w;
        }
        // Block factorisation over the node pairs {0,1} and {2,3}: the
        // leading block B by its adjugate, G = B^-1 C, the Schur complement
        // S = E - D G and its inverse.  Every principal block and Schur
        // complement of the element matrix keeps a positive definite
        // symmetric part (see k_dg_coef), and a 2x2 matrix with one has a
        // determinant at least that of its symmetric part, so both
        // determinants are positive: two reciprocals per cell, where the
        // scalar factorisation takes four in sequence.
        const double ib = recip(A[0][0] * A[1][1] - A[0][1] * A[1][0]);
        const double B00 = A[1][1] * ib, B01 = -A[0][1] * ib;
        const double B10 = -A[1][0] * ib, B11 = A[0][0] * ib;
        const double G00 = B00 * A[0][2] + B01 * A[1][2], G01 = B00 * A[0][3] + B01 * A[1][3];
        const double G10 = B10 * A[0][2] + B11 * A[1][2], G11 = B10 * A[0][3] + B11 * A[1][3];
        const double S00 = A[2][2] - (A[2][0] * G00 + A[2][1] * G10);
        const double S01 = A[2][3] - (A[2][0] * G01 + A[2][1] * G11);
        const double S10 = A[3][2] - (A[3][0] * G00 + A[3][1] * G10);
        const double S11 = A[3][3] - (A[3][0] * G01 + A[3][1] * G11);
        const double is = recip(S00 * S11 - S01 * S10);
        P[r][0] = B00; P[r][1] = B01; P[r][2] = B10; P[r][3] = B11;
        P[r][4] = A[2][0]; P[r][5] = A[2][1]; P[r][6] = A[3][0]; P[r][7] = A[3][1];
        P[r][8] = S11 * is; P[r][9] = -S01 * is; P[r][10] = -S10 * is; P[r][11] = S00 * is;
        P[r][12] = G00; P[r][13] = G01; P[r][14] = G10; P[r][15] = G11;
      }
    }
    if (live) {
      cp += CW;
      if (cp > hi) {
        ++cd;
        cp = cd < n_diag ? diag_lo(cd) : 0;
      }
    }
  };
  prepare(0);
  for (int k = 0; k < n_pad; ++k) {
    __syncthreads();  // traces of chunk k - 1 written, chunk k + 1 in its slot
    double x[Q][4];
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      // a face's two traces as one 16-byte word (neighbouring lanes hold
      // neighbouring cells: consecutive words, no bank conflicts)
      const double2 ux = reinterpret_cast<const double2*>(xf)[c_j[r]];
      const double2 uy = reinterpret_cast<const double2*>(yf)[c_i[r]];
      const double u0 = ux.x, u1 = ux.y, u2 = uy.x, u3 = uy.y;
      const double* Pr = P[r];
      if (TABLE) {
        x[r][0] = r0[r][0] + Pr[0] * u0 + Pr[1] * u1 + Pr[2] * u2 + Pr[3] * u3;
        x[r][1] = r0[r][1] + Pr[4] * u0 + Pr[5] * u1 + Pr[6] * u2 + Pr[7] * u3;
        x[r][2] = r0[r][2] + Pr[8] * u0 + Pr[9] * u1 + Pr[10] * u2 + Pr[11] * u3;
        x[r][3] = r0[r][3] + Pr[12] * u0 + Pr[13] * u1 + Pr[14] * u2 + Pr[15] * u3;
      } else {
        // F couples node (kx, ky) to the x-face traces only when kx is the
        // inflow column and to the y-face traces only when ky is the inflow
        // row: the other half of its entries are zero and are skipped
        double yv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double acc = r0[r][e];
          if ((e & 1) == (apos ? 0 : 1)) acc = acc + dmF[4 * e] * u0 + dmF[4 * e + 1] * u1;
          if ((e >> 1) == (bpos ? 0 : 1)) acc = acc + dmF[4 * e + 2] * u2 + dmF[4 * e + 3] * u3;
          yv[e] = acc;
        }
        // w = B^-1 y_top, z = y_bot - D w, x_bot = S^-1 z, x_top = w - G x_bot
        const double w0 = Pr[0] * yv[0] + Pr[1] * yv[1], w1 = Pr[2] * yv[0] + Pr[3] * yv[1];
        const double z0 = yv[2] - (Pr[4] * w0 + Pr[5] * w1);
        const double z1 = yv[3] - (Pr[6] * w0 + Pr[7] * w1);
        x[r][2] = Pr[8] * z0 + Pr[9] * z1;
        x[r][3] = Pr[10] * z0 + Pr[11] * z1;
        x[r][0] = w0 - (Pr[12] * x[r][2] + Pr[13] * x[r][3]);
        x[r][1] = w1 - (Pr[14] * x[r][2] + Pr[15] * x[r][3]);
      }
    }
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      if (!c_has[r]) continue;
      const double x0 = x[r][0], x1 = x[r][1], x2 = x[r][2], x3 = x[r][3];
      const int ci = c_i[r], cj = c_j[r];
      reinterpret_cast<double2*>(xf)[cj] = make_double2(apos ? x1 : x0, apos ? x3 : x2);
      reinterpret_cast<double2*>(yf)[ci] = make_double2(bpos ? x2 : x0, bpos ? x3 : x1);
      // outflow on a reflective downwind side, for the mirrored direction
      if (REFL && rx_out) {
        if (ci == (apos ? nx - 1 : 0)) {
          b_out[2 * cj] = apos ? x1 : x0;
          b_out[2 * cj + 1] = apos ? x3 : x2;
        }
      }
      if (REFL && ry_out) {
        if (cj == (bpos ? ny - 1 : 0)) {
          b_out[2 * ny + 2 * ci] = bpos ? x2 : x0;
          b_out[2 * ny + 2 * ci + 1] = bpos ? x3 : x1;
        }
      }
      // the plane is read once, by the direction sum: non-temporal stores
      double* po = reinterpret_cast<double*>(out + (c_pos[r] - lay_base));
      __builtin_nontemporal_store(x0, po);
      __builtin_nontemporal_store(x1, po + 1);
      __builtin_nontemporal_store(x2, po + 2);
      __builtin_nontemporal_store(x3, po + 3);
    }
    prepare((k + 1) & 1);
  }
  // Drain this wave's stores before the sweeping and loader paths join: the
  // compiler's wait counting cannot follow a mix of pending loads and stores,
  // and would otherwise wait for every load of the loader's ring.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

template <bool TABLE, int Q, bool REFL>
__global__ __launch_bounds__(512) void k_dg_sweep_pc(DgArgs g) {
  if (g.st->si.done) return;  // the whole workgroup: no barrier is left pending
  const int m = blockIdx.x;
  const bool apos = g.dir[3 * m + 0] > 0.0, bpos = g.dir[3 * m + 1] > 0.0;
  if (apos) {
    if (bpos) sweep_dir<TABLE, Q, REFL, true, true>(g);
    else sweep_dir<TABLE, Q, REFL, true, false>(g);
  } else {
    if (bpos) sweep_dir<TABLE, Q, REFL, false, true>(g);
    else sweep_dir<TABLE, Q, REFL, false, false>(g);
  }
}

size_t dg_sweep_lds_bytes(bool table, int cw, int n_mat, int nx, int ny) {
  return sizeof(double) * ((size_t)2 * cw * 5 + (table ? (size_t)n_mat * kDgRow : 0) +
                           (size_t)2 * (nx + ny));
}

hipError_t launch_si_start(const DgArgs& a, int si_max, hipStream_t s) {
  const long long nc = (long long)a.nx * a.ny;
  long long b = (nc + 255) / 256;
  const int grid = (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
  const long long nb = a.bnd ? (long long)a.n_dir * 2 * (a.nx + a.ny) : 0;
  hipLaunchKernelGGL(k_si_start, dim3(grid), dim3(256), 0, s, a.nx, a.ny, a.sig_s,
                     a.phi_post, a.phi_c, a.src, a.bnd ? a.bnd + nb : nullptr, nb, a.st, si_max);
  return hipGetLastError();
}

__global__ void k_si_check(DevState* st) {
  if (threadIdx.x == 0 && !st->halt && !st->si.done) {
    st->halt = 1;
    st->si.done = 1;
  }
}

__global__ void k_dsa_check(DevState* st) {
  if (threadIdx.x == 0 && !st->halt && !st->si.done && !st->dsa.done) {
    st->halt = 1;
    st->si.done = 1;
  }
}

hipError_t launch_dsa_check(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_dsa_check, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_si_check(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_si_check, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_dg_sweep(const DgArgs& a, bool table, hipStream_t s) {
  const size_t lds = dg_sweep_lds_bytes(table, a.cw, a.n_mat, a.nx, a.ny);
  const int q = a.cells_per_lane;  // cells per sweeping and per loader lane
  if ((q != 1 && q != 2 && q != 4) || a.cw % (64 * q) || a.cw / (64 * q) > 4)
    return hipErrorInvalidValue;
  const dim3 block(2 * a.cw / q);  // as many loader waves as sweeping waves
  const bool refl = a.bc != 0 && a.bnd != nullptr;
#define SLH_DG_SWEEP(T_, Q_)                                                                  \
  do {                                                                                        \
    if (refl) hipLaunchKernelGGL((k_dg_sweep_pc<T_, Q_, true>), dim3(a.n_dir), block, lds, s, a); \
    else hipLaunchKernelGGL((k_dg_sweep_pc<T_, Q_, false>), dim3(a.n_dir), block, lds, s, a);     \
  } while (0)
  if (table) {
    if (q == 1) SLH_DG_SWEEP(true, 1);
    else if (q == 2) SLH_DG_SWEEP(true, 2);
    else SLH_DG_SWEEP(true, 4);
  } else {
    if (q == 1) SLH_DG_SWEEP(false, 1);
    else if (q == 2) SLH_DG_SWEEP(false, 2);
    else SLH_DG_SWEEP(false, 4);
  }
#undef SLH_DG_SWEEP
  return hipGetLastError();
}

// The reduction of a source iteration, in two kernels.  k_dg_famsum: at
// every node of each layout, the sum of w_m psi_m over that layout's
// directions in their order (every plane read once, in whole cache lines).
// k_dg_combine, per row-major cell: phi_new = sum over layout A + sum over
// layout B, in place (the sweep read only S); the next iterate's nodal source
// S = sigma_s/(4 pi) (phi_new + phi_post) in both layouts (unused when the
// iteration stops here); block partials of |phi_new - phi_old|^2 and
// |phi_new|^2, or |phi_new + phi_pre + phi_post|^2 when phi_pre is given (the
// step's whole flux as the reference of the stopping test).  With the
// diffusion correction the combine keeps phi_new - phi_old in dnode instead
// and leaves the source and the residual to k_dsa_apply.
constexpr int kRedBlock = 256;

int dg_reduce_partials(long long n_nodes) {
  long long b = (n_nodes + kRedBlock - 1) / kRedBlock;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

__global__ __launch_bounds__(kRedBlock) void k_dg_famsum(
    const int* __restrict__ fam_dirs, int n_a, int n_dir, long long n_nodes,
    const double* __restrict__ psi, const double* __restrict__ dir,
    double* __restrict__ phi_fam, const DevState* st) {
  if (st->si.done) return;
  // the first half of the grid sums layout A, the second layout B
  const int half = (int)(gridDim.x >> 1);
  const bool fb = (int)blockIdx.x >= half;
  const int u0 = fb ? n_a : 0, u1 = fb ? n_dir : n_a;
  double2* __restrict__ out = reinterpret_cast<double2*>(phi_fam + (fb ? n_nodes : 0));
  // two nodes per thread (16-byte loads; n_nodes = 4 cells is even)
  const long long n2 = n_nodes >> 1;
  for (long long k = (long long)(blockIdx.x - (fb ? half : 0)) * kRedBlock + threadIdx.x;
       k < n2; k += (long long)half * kRedBlock) {
    // sixteen planes' loads in flight per step, added in direction order
    double vx = 0.0, vy = 0.0;
    int u = u0;
    for (; u + 16 <= u1; u += 16) {
      double2 t[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {  // read once: non-temporal loads
        const double* pp = psi + (long long)fam_dirs[u + e] * n_nodes + 2 * k;
        t[e].x = __builtin_nontemporal_load(pp);
        t[e].y = __builtin_nontemporal_load(pp + 1);
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const double w = dir[3 * fam_dirs[u + e] + 2];
        vx += w * t[e].x;
        vy += w * t[e].y;
      }
    }
    for (; u < u1; ++u) {
      const int m = fam_dirs[u];
      const double2 t = reinterpret_cast<const double2*>(psi + (long long)m * n_nodes)[k];
      vx += dir[3 * m + 2] * t.x;
      vy += dir[3 * m + 2] * t.y;
    }
    out[k] = make_double2(vx, vy);
  }
}

// Partials of a block: tree sum of the threads' values in a fixed order.
__device__ __forceinline__ void block_partials(double dsum, double nsum, double* partials) {
  __shared__ double s_d[kRedBlock], s_n[kRedBlock];
  s_d[threadIdx.x] = dsum;
  s_n[threadIdx.x] = nsum;
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_d[threadIdx.x] += s_d[threadIdx.x + off];
      s_n[threadIdx.x] += s_n[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s_d[0];
    partials[2 * blockIdx.x + 1] = s_n[0];
  }
}

// The next iterate's nodal source of cell (ci, cj) in both layouts, and the
// cell's contribution to the stopping test.
__device__ __forceinline__ void next_source(int nx, int ny, long long c,
                                            double4 v, double4 d, double ssc, double pp,
                                            const double* phi_pre, double* S, double& dsum,
                                            double& nsum) {
  const long long n = (long long)nx * ny;
  const int ci = (int)(c % nx), cj = (int)(c / nx);
  const double4 sv = make_double4(ssc * (v.x + pp), ssc * (v.y + pp), ssc * (v.z + pp),
                                  ssc * (v.w + pp));
  reinterpret_cast<double4*>(S)[lay_pos(nx, ny, ci, cj, true)] = sv;
  reinterpret_cast<double4*>(S)[n + lay_pos(nx, ny, ci, cj, false)] = sv;
  const double r = phi_pre ? phi_pre[c] + pp : 0.0;
  dsum += d.x * d.x + d.y * d.y + d.z * d.z + d.w * d.w;
  nsum += (v.x + r) * (v.x + r) + (v.y + r) * (v.y + r) + (v.z + r) * (v.z + r) +
          (v.w + r) * (v.w + r);
}

__global__ __launch_bounds__(kRedBlock) void k_dg_combine(
    int nx, int ny, const double* __restrict__ phi_fam,
    double* __restrict__ phi, const double* __restrict__ sig_s,
    const double* __restrict__ phi_post, const double* __restrict__ phi_pre,
    double* __restrict__ S, double* __restrict__ partials, double* __restrict__ dnode,
    const DevState* st) {
  if (st->si.done) return;
  const double inv4pi = 0.25 / M_PI;
  const long long n = (long long)nx * ny;
  const double4* fam = reinterpret_cast<const double4*>(phi_fam);
  double dsum = 0.0, nsum = 0.0;
  for (long long c = (long long)blockIdx.x * kRedBlock + threadIdx.x; c < n;
       c += (long long)gridDim.x * kRedBlock) {
    const int ci = (int)(c % nx), cj = (int)(c / nx);
    const double4 a = fam[lay_pos(nx, ny, ci, cj, true)];
    const double4 b = fam[n + lay_pos(nx, ny, ci, cj, false)];
    const double4 v = make_double4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
    const double4 o = reinterpret_cast<const double4*>(phi)[c];
    const double4 d = make_double4(v.x - o.x, v.y - o.y, v.z - o.z, v.w - o.w);
    reinterpret_cast<double4*>(phi)[c] = v;
    if (dnode) {  // the correction, the source and the residual come later
      reinterpret_cast<double4*>(dnode)[c] = d;
      continue;
    }
    next_source(nx, ny, c, v, d, sig_s[c] * inv4pi, phi_post[c], phi_pre, S, dsum, nsum);
  }
  if (dnode) return;  // the same for the whole grid
  block_partials(dsum, nsum, partials);
}

// phi += delta (per cell) at every node, the next source, and partials of
// |dnode + delta|^2 and |phi|^2 (or of the whole-flux norm) for k_dg_residual.
__global__ __launch_bounds__(kRedBlock) void k_dsa_apply(
    int nx, int ny, double* __restrict__ phi,
    const double* __restrict__ dnode, const double* __restrict__ delta,
    const double* __restrict__ sig_s, const double* __restrict__ phi_post,
    const double* __restrict__ phi_pre, double* __restrict__ S, double* __restrict__ partials,
    const DevState* st) {
  if (st->si.done) return;
  const double inv4pi = 0.25 / M_PI;
  const long long n = (long long)nx * ny;
  double dsum = 0.0, nsum = 0.0;
  for (long long c = (long long)blockIdx.x * kRedBlock + threadIdx.x; c < n;
       c += (long long)gridDim.x * kRedBlock) {
    const double dl = delta[c];
    const double4 o = reinterpret_cast<const double4*>(phi)[c];
    const double4 dn = reinterpret_cast<const double4*>(dnode)[c];
    const double4 v = make_double4(o.x + dl, o.y + dl, o.z + dl, o.w + dl);
    const double4 d = make_double4(dn.x + dl, dn.y + dl, dn.z + dl, dn.w + dl);
    reinterpret_cast<double4*>(phi)[c] = v;
    next_source(nx, ny, c, v, d, sig_s[c] * inv4pi, phi_post[c], phi_pre, S, dsum, nsum);
  }
  block_partials(dsum, nsum, partials);
}

// Sums the block partials with a fixed association order (strided
// per-thread sums, then a tree) and takes the iteration's decision: done
// when |phi_new - phi_old| <= tol |phi_new| (converged), when the iteration
// limit is reached, or when the residual is not finite.  After a diffusion
// correction (dsa) it also books that correction's conjugate-gradient
// iterations and whether they reached their tolerance.
__global__ __launch_bounds__(256) void k_dg_residual(const double* partials, int n_part,
                                                     DevState* st, double si_tol, int si_max,
                                                     int dsa) {
  if (st->si.done) return;
  __shared__ double s_d[256], s_n[256];
  double d = 0.0, n = 0.0;
  for (int b = threadIdx.x; b < n_part; b += 256) {
    d += partials[2 * b];
    n += partials[2 * b + 1];
  }
  s_d[threadIdx.x] = d;
  s_n[threadIdx.x] = n;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_d[threadIdx.x] += s_d[threadIdx.x + off];
      s_n[threadIdx.x] += s_n[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double dn2 = s_d[0], nrm2 = s_n[0];
    const double dn = sqrt(dn2), nrm = sqrt(nrm2);
    st->si.dn2_prev = st->si.iter > 0 ? st->si.dn2 : 0.0;
    st->si.dn2 = dn2;
    st->si.nrm2 = nrm2;
    st->si.iter += 1;
    const int bad = !isfinite(dn) || !isfinite(nrm);
    const int conv = !bad && dn <= si_tol * nrm;
    st->si.bad = bad;
    st->si.conv = conv;
    st->si.done = bad || conv || st->si.iter >= si_max;
    if (dsa) {
      st->dsa_corrections += 1;
      st->dsa_iter_total += st->dsa.iter;
      if (st->dsa.iter > st->dsa_iter_max) st->dsa_iter_max = st->dsa.iter;
      if (!st->dsa.conv) st->dsa_unconv += 1;
    }
  }
}

hipError_t launch_dg_reduce(const DgArgs& a, double* partials, int n_part, double si_tol,
                            int si_max, hipStream_t s) {
  const long long n_nodes = 4ll * a.nx * a.ny;
  hipLaunchKernelGGL(k_dg_famsum, dim3(2 * dg_reduce_partials(n_nodes / 2)), dim3(kRedBlock), 0, s,
                     a.fam_dirs, a.fam_n, a.n_dir, n_nodes, (const double*)a.psi, a.dir,
                     a.phi_fam, (const DevState*)a.st);
  hipLaunchKernelGGL(k_dg_combine, dim3(n_part), dim3(kRedBlock), 0, s, a.nx, a.ny,
                     (const double*)a.phi_fam, a.phi_c, a.sig_s, a.phi_post, a.phi_pre, a.src,
                     partials, a.dnode, (const DevState*)a.st);
  if (!a.dnode)
    hipLaunchKernelGGL(k_dg_residual, dim3(1), dim3(256), 0, s, (const double*)partials, n_part,
                       a.st, si_tol, si_max, 0);
  return hipGetLastError();
}

hipError_t launch_dsa_apply(const DgArgs& a, const double* delta, double* partials, int n_part,
                            double si_tol, int si_max, hipStream_t s) {
  hipLaunchKernelGGL(k_dsa_apply, dim3(n_part), dim3(kRedBlock), 0, s, a.nx, a.ny,
                     a.phi_c, (const double*)a.dnode, delta, a.sig_s, a.phi_post, a.phi_pre,
                     a.src, partials, (const DevState*)a.st);
  hipLaunchKernelGGL(k_dg_residual, dim3(1), dim3(256), 0, s, (const double*)partials, n_part,
                     a.st, si_tol, si_max, 1);
  return hipGetLastError();
}

}  // namespace slh
