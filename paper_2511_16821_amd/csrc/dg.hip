// Collided solve of the hybrid step (step 2 of Sec. 2.2): discrete ordinates
// with bilinear discontinuous Galerkin in space, upwind faces, vacuum inflow,
// and a step-averaged time closure sigma_e = sigma_t + tau/(c dt).  One
// transport sweep per direction and source-iteration sweep.
//
// Device layout: one workgroup per direction.  The workgroup walks the cells
// in diagonal wavefronts of its quadrant's upwind order; cells on one diagonal
// have distinct rows and columns, so the outflow traces they hand to the next
// diagonal live in two small LDS arrays (one trace per row for the x faces,
// one per column for the y faces).  Each cell solves its 4x4 system in
// registers.  The weighted nodal solution w_m psi_m goes to a per-direction
// plane, and the directions are summed in a fixed order by a second kernel,
// so the scalar flux does not depend on scheduling.
//
// Element matrices on a cell of size hx x hy, node k = kx + 2 ky at
// (x_kx, y_ky), 1-D factors  M = h/6 [[2,1],[1,2]] (mass) and
// K = 1/2 [[-1,1],[-1,1]] (K[i][j] = int L_i L_j'):
//   A = a Kx(x)My + b Mx(x)Ky + sig_e Mx(x)My
//     + |a| (e_f e_f^T)(x)My + |b| Mx(x)(e_g e_g^T)
// where f (g) is the local index of the x (y) inflow face; the right side is
// (Mx(x)My) S + |a| e_f (x) My up_x + |b| Mx up_y (x) e_g with the upwind
// traces up_x, up_y (zero on the domain boundary).
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

// Gaussian elimination without pivoting.  The upwind element matrix has a
// positive-definite symmetric part (mass and inflow terms are SPD, the
// streaming term's symmetric part is the outflow-minus-inflow face mass,
// which the inflow term turns into |Omega.n| on every face), so every
// leading block is invertible and no pivot vanishes.  Each pivot's
// reciprocal is formed once and reused in the back substitution.
__device__ __forceinline__ void solve4(double A[4][4], double r[4], double x[4]) {
  double inv[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    inv[c] = recip(A[c][c]);
#pragma unroll
    for (int i = c + 1; i < 4; ++i) {
      const double f = A[i][c] * inv[c];
#pragma unroll
      for (int k = c + 1; k < 4; ++k) A[i][k] -= f * A[c][k];
      r[i] -= f * r[c];
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    double v = r[i];
#pragma unroll
    for (int k = i + 1; k < 4; ++k) v -= A[i][k] * x[k];
    x[i] = v * inv[i];
  }
}

// Nodal source of the collided equation for the current iterate:
// S = sigma_s/(4 pi) (phi_c + phi_post), once per source iteration.
__global__ void k_dg_source(long long n, const double* __restrict__ sig_s,
                            const double* __restrict__ phi_post,
                            const double* __restrict__ phi_in, double* __restrict__ S) {
  const double inv4pi = 0.25 / M_PI;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double ssc = sig_s[i] * inv4pi;
    const double pp = phi_post[i];
    const double4 f = reinterpret_cast<const double4*>(phi_in)[i];
    reinterpret_cast<double4*>(S)[i] = make_double4(ssc * (f.x + pp), ssc * (f.y + pp),
                                                    ssc * (f.z + pp), ssc * (f.w + pp));
  }
}

__global__ __launch_bounds__(256) void k_dg_sweep(DgArgs g) {
  extern __shared__ double s_face[];  // [ny][2] x-traces, then [nx][2] y-traces
  const int m = blockIdx.x;
  const double a = g.dir[3 * m + 0], b = g.dir[3 * m + 1], wm = g.dir[3 * m + 2];
  const int nx = g.nx, ny = g.ny;
  double* xf = s_face;
  double* yf = s_face + 2 * ny;
  for (int k = threadIdx.x; k < 2 * (nx + ny); k += blockDim.x) s_face[k] = 0.0;
  __syncthreads();

  const double hx = g.hx, hy = g.hy;
  const bool apos = a > 0.0, bpos = b > 0.0;
  const int fx = apos ? 0 : 1, fy = bpos ? 0 : 1;
  const double aa = fabs(a), ab = fabs(b);
  const double Mx[2][2] = {{hx / 3.0, hx / 6.0}, {hx / 6.0, hx / 3.0}};
  const double My[2][2] = {{hy / 3.0, hy / 6.0}, {hy / 6.0, hy / 3.0}};
  const double K[2][2] = {{-0.5, 0.5}, {-0.5, 0.5}};
  // direction-only part of the element matrix (uniform mesh)
  double A0[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int kx = k & 1, ky = k >> 1;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int lx = l & 1, ly = l >> 1;
      double v = a * K[kx][lx] * My[ky][ly] + b * Mx[kx][lx] * K[ky][ly];
      if (kx == fx && lx == fx) v += aa * My[ky][ly];
      if (ky == fy && ly == fy) v += ab * Mx[kx][lx];
      A0[k][l] = v;
    }
  }
  const double4* __restrict__ S4 = reinterpret_cast<const double4*>(g.src);
  double4* __restrict__ out = reinterpret_cast<double4*>(g.psi + (long long)m * 4 * nx * ny);

  const int n_diag = nx + ny - 1;
  const int tid = threadIdx.x, B = blockDim.x;
  // prefetch of the first cell of this thread on the next diagonal
  int p_ip = tid;  // diagonal 0 holds ip = 0 only
  bool p_has = p_ip <= 0;
  double p_se = 0.0;
  double4 p_S = make_double4(0.0, 0.0, 0.0, 0.0);
  long long p_cell = 0;
  if (p_has) {
    const int i = apos ? 0 : nx - 1, j = bpos ? 0 : ny - 1;
    p_cell = (long long)j * nx + i;
    p_se = g.sig_e[p_cell];
    p_S = S4[p_cell];
  }
  for (int d = 0; d < n_diag; ++d) {
    const int i_lo = d - (ny - 1) > 0 ? d - (ny - 1) : 0;
    const int i_hi = d < nx - 1 ? d : nx - 1;
    int ip = p_ip;
    bool has = p_has;
    double se = p_se;
    double4 Sv = p_S;
    long long cell = p_cell;
    if (d + 1 < n_diag) {  // issue next diagonal's loads before this one's work
      const int dn = d + 1;
      const int lo_n = dn - (ny - 1) > 0 ? dn - (ny - 1) : 0;
      const int hi_n = dn < nx - 1 ? dn : nx - 1;
      p_ip = lo_n + tid;
      p_has = p_ip <= hi_n;
      if (p_has) {
        const int jp = dn - p_ip;
        const int i = apos ? p_ip : nx - 1 - p_ip, j = bpos ? jp : ny - 1 - jp;
        p_cell = (long long)j * nx + i;
        p_se = g.sig_e[p_cell];
        p_S = S4[p_cell];
      }
    }
    for (;;) {
      if (!has) break;
      const int jp = d - ip;
      const int i = apos ? ip : nx - 1 - ip;
      const int j = bpos ? jp : ny - 1 - jp;
      const double S[4] = {Sv.x, Sv.y, Sv.z, Sv.w};
      const double upx0 = xf[2 * j], upx1 = xf[2 * j + 1];
      const double upy0 = yf[2 * i], upy1 = yf[2 * i + 1];
      double A[4][4], r[4], x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int kx = k & 1, ky = k >> 1;
        double rk = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const int lx = l & 1, ly = l >> 1;
          const double mm = Mx[kx][lx] * My[ky][ly];
          A[k][l] = A0[k][l] + se * mm;
          rk += mm * S[l];
        }
        if (kx == fx) rk += aa * (My[ky][0] * upx0 + My[ky][1] * upx1);
        if (ky == fy) rk += ab * (Mx[kx][0] * upy0 + Mx[kx][1] * upy1);
        r[k] = rk;
      }
      solve4(A, r, x);
      // outflow traces for the downstream neighbours
      xf[2 * j] = apos ? x[1] : x[0];
      xf[2 * j + 1] = apos ? x[3] : x[2];
      yf[2 * i] = bpos ? x[2] : x[0];
      yf[2 * i + 1] = bpos ? x[3] : x[1];
      out[cell] = make_double4(wm * x[0], wm * x[1], wm * x[2], wm * x[3]);
      // further cells of this thread on a diagonal longer than the block
      ip += B;
      has = ip <= i_hi;
      if (has) {
        const int jq = d - ip;
        const int iq = apos ? ip : nx - 1 - ip, jj = bpos ? jq : ny - 1 - jq;
        cell = (long long)jj * nx + iq;
        se = g.sig_e[cell];
        Sv = S4[cell];
      }
    }
    (void)i_lo;
    __syncthreads();
  }
}

hipError_t launch_dg_sweep(const DgArgs& a, hipStream_t s) {
  const long long nc = (long long)a.nx * a.ny;
  long long b = (nc + 255) / 256;
  const int grid = (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
  hipLaunchKernelGGL(k_dg_source, dim3(grid), dim3(256), 0, s, nc, a.sig_s, a.phi_post,
                     a.phi_in, a.src);
  const size_t lds = sizeof(double) * 2 * (size_t)(a.nx + a.ny);
  hipLaunchKernelGGL(k_dg_sweep, dim3(a.n_dir), dim3(256), lds, s, a);
  return hipGetLastError();
}

// phi_new[k] = sum_m psi[m][k] in direction order; block partials of
// |phi_new - phi_old|^2 and |phi_new|^2.
constexpr int kRedBlock = 256;

int dg_reduce_partials(long long n_nodes) {
  long long b = (n_nodes + kRedBlock - 1) / kRedBlock;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

__global__ __launch_bounds__(kRedBlock) void k_dg_reduce(int n_dir, long long n_nodes,
                                                         const double* __restrict__ psi,
                                                         const double* __restrict__ phi_old,
                                                         double* __restrict__ phi_new,
                                                         double* __restrict__ partials) {
  __shared__ double s_d[kRedBlock], s_n[kRedBlock];
  double dsum = 0.0, nsum = 0.0;
  for (long long k = (long long)blockIdx.x * kRedBlock + threadIdx.x; k < n_nodes;
       k += (long long)gridDim.x * kRedBlock) {
    double v = 0.0;
    for (int m = 0; m < n_dir; ++m) v += psi[(long long)m * n_nodes + k];
    const double d = v - phi_old[k];
    phi_new[k] = v;
    dsum += d * d;
    nsum += v * v;
  }
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

// Sums the block partials into partials[2*n_part .. +1] with a fixed
// association order (strided per-thread sums, then a tree).
__global__ __launch_bounds__(256) void k_dg_residual(double* partials, int n_part) {
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
    partials[2 * n_part] = s_d[0];
    partials[2 * n_part + 1] = s_n[0];
  }
}

hipError_t launch_dg_reduce(int n_dir, long long n_nodes, const double* psi,
                            const double* phi_old, double* phi_new, double* partials,
                            int n_part, hipStream_t s) {
  hipLaunchKernelGGL(k_dg_reduce, dim3(n_part), dim3(kRedBlock), 0, s, n_dir, n_nodes, psi,
                     phi_old, phi_new, partials);
  hipLaunchKernelGGL(k_dg_residual, dim3(1), dim3(256), 0, s, partials, n_part);
  return hipGetLastError();
}

}  // namespace slh
