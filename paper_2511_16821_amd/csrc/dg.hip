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

__device__ __forceinline__ void solve4(double A[4][4], double r[4], double x[4]) {
  // Gauss-Jordan elimination with row pivoting on the 4x4 element system.
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int p = c;
#pragma unroll
    for (int i = c + 1; i < 4; ++i)
      if (fabs(A[i][c]) > fabs(A[p][c])) p = i;
    if (p != c) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double t = A[c][k]; A[c][k] = A[p][k]; A[p][k] = t;
      }
      const double t = r[c]; r[c] = r[p]; r[p] = t;
    }
    const double inv = 1.0 / A[c][c];
#pragma unroll
    for (int k = 0; k < 4; ++k) A[c][k] *= inv;
    r[c] *= inv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i == c) continue;
      const double f = A[i][c];
#pragma unroll
      for (int k = 0; k < 4; ++k) A[i][k] -= f * A[c][k];
      r[i] -= f * r[c];
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = r[k];
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
  const int fx = a > 0.0 ? 0 : 1, fy = b > 0.0 ? 0 : 1;
  const double aa = fabs(a), ab = fabs(b);
  const double Mx[2][2] = {{hx / 3.0, hx / 6.0}, {hx / 6.0, hx / 3.0}};
  const double My[2][2] = {{hy / 3.0, hy / 6.0}, {hy / 6.0, hy / 3.0}};
  const double K[2][2] = {{-0.5, 0.5}, {-0.5, 0.5}};
  const double inv4pi = 0.25 / M_PI;
  double* psi_m = g.psi + (long long)m * 4 * nx * ny;

  const int n_diag = nx + ny - 1;
  for (int d = 0; d < n_diag; ++d) {
    const int i_lo = d - (ny - 1) > 0 ? d - (ny - 1) : 0;
    const int i_hi = d < nx - 1 ? d : nx - 1;
    for (int ip = i_lo + (int)threadIdx.x; ip <= i_hi; ip += blockDim.x) {
      const int jp = d - ip;
      const int i = a > 0.0 ? ip : nx - 1 - ip;
      const int j = b > 0.0 ? jp : ny - 1 - jp;
      const long long cell = (long long)j * nx + i;
      const double se = g.sig_e[cell];
      const double ssc = g.sig_s[cell] * inv4pi;
      const double pp = g.phi_post[cell];
      double S[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) S[k] = ssc * (g.phi_in[4 * cell + k] + pp);
      const double upx[2] = {xf[2 * j], xf[2 * j + 1]};
      const double upy[2] = {yf[2 * i], yf[2 * i + 1]};
      double A[4][4], r[4], x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int kx = k & 1, ky = k >> 1;
        double rk = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const int lx = l & 1, ly = l >> 1;
          const double mm = Mx[kx][lx] * My[ky][ly];
          double v = a * K[kx][lx] * My[ky][ly] + b * Mx[kx][lx] * K[ky][ly] + se * mm;
          if (kx == fx && lx == fx) v += aa * My[ky][ly];
          if (ky == fy && ly == fy) v += ab * Mx[kx][lx];
          A[k][l] = v;
          rk += mm * S[l];
        }
        if (kx == fx) rk += aa * (My[ky][0] * upx[0] + My[ky][1] * upx[1]);
        if (ky == fy) rk += ab * (Mx[kx][0] * upy[0] + Mx[kx][1] * upy[1]);
        r[k] = rk;
      }
      solve4(A, r, x);
      // outflow traces for the downstream neighbours
      const int ox = 1 - fx, oy = 1 - fy;
      xf[2 * j] = x[ox];
      xf[2 * j + 1] = x[ox + 2];
      yf[2 * i] = x[2 * oy];
      yf[2 * i + 1] = x[2 * oy + 1];
#pragma unroll
      for (int k = 0; k < 4; ++k) psi_m[4 * cell + k] = wm * x[k];
    }
    __syncthreads();
  }
}

hipError_t launch_dg_sweep(const DgArgs& a, hipStream_t s) {
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

// Sums the block partials in block order into partials[2*n_part .. +1].
__global__ void k_dg_residual(double* partials, int n_part) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double d = 0.0, n = 0.0;
  for (int b = 0; b < n_part; ++b) {
    d += partials[2 * b];
    n += partials[2 * b + 1];
  }
  partials[2 * n_part] = d;
  partials[2 * n_part + 1] = n;
}

hipError_t launch_dg_reduce(int n_dir, long long n_nodes, const double* psi,
                            const double* phi_old, double* phi_new, double* partials,
                            int n_part, hipStream_t s) {
  hipLaunchKernelGGL(k_dg_reduce, dim3(n_part), dim3(kRedBlock), 0, s, n_dir, n_nodes, psi,
                     phi_old, phi_new, partials);
  hipLaunchKernelGGL(k_dg_residual, dim3(1), dim3(64), 0, s, partials, n_part);
  return hipGetLastError();
}

}  // namespace slh
