// Diffusion closing stage: the collided flux of step 2 of Sec. 2.2 from a
// cell-centred finite-volume diffusion equation (the cheap deterministic
// solver the paper suggests in place of S_N),
//   sigma_r phi - div(D grad phi) = sigma_s phi_post,
//   sigma_r = sigma_a + tau/(c dt),  D = 1/(3 (sigma_t + tau/(c dt)))
// (no tau/(c dt) in steady state), harmonic-mean face coefficients, Marshak
// vacuum sides and zero-current reflective sides.  The symmetric positive
// definite system is solved by Jacobi-preconditioned conjugate gradients
// from phi = 0, each iteration three kernels:
//   k_cg_spmv:     p_k = z + beta p_{k-1} (every cell also forms its four
//                  neighbours' p_k, so the update needs no separate pass),
//                  q = A p_k, block partials of p_k . q;
//   k_cg_update:   alpha = rz / (p_k . q) (each block sums the partials in
//                  the same fixed order), x += alpha p_k, r -= alpha q,
//                  z = r / diag, block partials of r . z and r . r;
//   k_cg_residual: one block: beta, the stopping test ||r|| <= tol ||b||,
//                  the iteration count, in the source-iteration state, so the
//                  host loop and the graph batching of the S_N path apply.
// Reductions use fixed association orders: results do not depend on
// scheduling.  The two p buffers alternate by iteration parity.  Meshes of
// up to 4096 cells run the whole solve in one workgroup instead
// (k_cg_solve_one_block), with barriers in place of launches: there the
// launches cost more than the work (a 1500-cell solve of 279 iterations
// 2.4 ms against 4.4 ms), while on larger meshes one compute unit's share of
// the bandwidth is the limit (19600 cells: 1.8 against 1.1 ms per step).
#include "slh_common.hpp"

namespace slh {

constexpr int kCgBlock = 256;

int cg_partials(long long n) {
  long long b = (n + kCgBlock - 1) / kCgBlock;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

// Per-cell coefficients: diagonal, coupling to the x+1 neighbour (cE) and to
// the y+1 neighbour (cN), zero across the domain boundary.
__global__ void k_diff_coef(int nx, int ny, const double2* __restrict__ mat, double tt,
                            double hx, double hy, int bc, double* __restrict__ diag,
                            double* __restrict__ cE, double* __restrict__ cN) {
  const long long n = (long long)nx * ny;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(k % nx), j = (int)(k / nx);
    const double2 m = mat[k];  // (sigma_s, sigma_a)
    const double D = 1.0 / (3.0 * (m.y + m.x + tt));
    double d = m.y + tt;
    double e = 0.0, no = 0.0;
    // x faces
    if (i + 1 < nx) {
      const double2 mn = mat[k + 1];
      const double Dn = 1.0 / (3.0 * (mn.y + mn.x + tt));
      e = 2.0 * D * Dn / (D + Dn) / (hx * hx);
      d += e;
    } else if (!(bc & 2)) {
      d += 2.0 * D / (hx * (hx + 4.0 * D));
    }
    if (i > 0) {
      const double2 mw = mat[k - 1];
      const double Dw = 1.0 / (3.0 * (mw.y + mw.x + tt));
      d += 2.0 * Dw * D / (Dw + D) / (hx * hx);
    } else if (!(bc & 1)) {
      d += 2.0 * D / (hx * (hx + 4.0 * D));
    }
    // y faces
    if (j + 1 < ny) {
      const double2 mn = mat[k + nx];
      const double Dn = 1.0 / (3.0 * (mn.y + mn.x + tt));
      no = 2.0 * D * Dn / (D + Dn) / (hy * hy);
      d += no;
    } else if (!(bc & 8)) {
      d += 2.0 * D / (hy * (hy + 4.0 * D));
    }
    if (j > 0) {
      const double2 ms = mat[k - nx];
      const double Ds = 1.0 / (3.0 * (ms.y + ms.x + tt));
      d += 2.0 * Ds * D / (Ds + D) / (hy * hy);
    } else if (!(bc & 4)) {
      d += 2.0 * D / (hy * (hy + 4.0 * D));
    }
    diag[k] = d;
    cE[k] = e;
    cN[k] = no;
  }
}

hipError_t launch_diff_coef(int nx, int ny, const double2* mat, double tt, double hx, double hy,
                            int bc, double* diag, double* cE, double* cN, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_diff_coef, dim3(cg_partials(n)), dim3(kCgBlock), 0, s, nx, ny, mat, tt,
                     hx, hy, bc, diag, cE, cN);
  return hipGetLastError();
}

// Block sum of two values per thread into out[2 blockIdx.x + {0,1}].
__device__ __forceinline__ void block_sum2(double a, double b, double* out) {
  __shared__ double s_a[kCgBlock], s_b[kCgBlock];
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  for (int off = kCgBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_a[threadIdx.x] += s_a[threadIdx.x + off];
      s_b[threadIdx.x] += s_b[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = s_a[0];
    out[2 * blockIdx.x + 1] = s_b[0];
  }
}

// Fixed-order sum of the first (w = 0) or second (w = 1) value of n_part
// block partials; every thread of the block gets the result.
__device__ __forceinline__ double sum_partials(const double* part, int n_part, int w) {
  __shared__ double s[kCgBlock];
  double v = 0.0;
  for (int b = threadIdx.x; b < n_part; b += kCgBlock) v += part[2 * b + w];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = kCgBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

// Start: b = sigma_s phi_post, x = 0, r = b, z = r / diag, p_{-1} = 0
// (buffer 1), partials of r . z and b . b.
__global__ __launch_bounds__(kCgBlock) void k_cg_start(
    long long n, const double* __restrict__ sig_s, const double* __restrict__ phi_post,
    const double* __restrict__ diag, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ z, double* __restrict__ p1, double* __restrict__ part,
    const int* halt) {
  if (*halt) return;
  double rz = 0.0, bb = 0.0;
  for (long long k = (long long)blockIdx.x * kCgBlock + threadIdx.x; k < n;
       k += (long long)gridDim.x * kCgBlock) {
    const double b = sig_s[k] * phi_post[k];
    const double zk = b / diag[k];
    x[k] = 0.0;
    r[k] = b;
    z[k] = zk;
    p1[k] = 0.0;
    rz += b * zk;
    bb += b * b;
  }
  block_sum2(rz, bb, part);
}

__global__ __launch_bounds__(kCgBlock) void k_cg_start_state(const double* part, int n_part,
                                                             IterState* cs, const int* gate,
                                                             int max_iter, const int* halt) {
  if ((gate && *gate) || (halt && *halt)) return;
  const double rz = sum_partials(part, n_part, 0);
  const double bb = sum_partials(part, n_part, 1);
  if (threadIdx.x == 0) {
    cs->iter = 0;
    cs->bad = 0;
    cs->rz = rz;
    cs->beta = 0.0;
    cs->bb = bb;
    cs->dn2 = bb;
    cs->dn2_prev = 0.0;
    cs->nrm2 = bb;
    // a zero source has the exact solution 0
    const int conv = max_iter == 0 || bb == 0.0;
    cs->conv = conv;
    cs->done = conv;
    if (bb == 0.0) cs->dn2 = 0.0;
  }
}

// Start of the diffusion correction of a source iteration: b = sigma_s times
// the cell average of phi^{k+1/2} - phi^k (dnode, four nodes per cell), x = 0,
// r = b, z = r / diag, p_{-1} = 0, partials of r . z and b . b.
__global__ __launch_bounds__(kCgBlock) void k_dsa_start(
    long long n, const double* __restrict__ sig_s, const double* __restrict__ dnode,
    const double* __restrict__ diag, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ z, double* __restrict__ p1, double* __restrict__ part,
    const int* gate) {
  if (*gate) return;
  double rz = 0.0, bb = 0.0;
  for (long long k = (long long)blockIdx.x * kCgBlock + threadIdx.x; k < n;
       k += (long long)gridDim.x * kCgBlock) {
    const double4 d = reinterpret_cast<const double4*>(dnode)[k];
    const double b = sig_s[k] * (0.25 * ((d.x + d.y) + (d.z + d.w)));
    const double zk = b / diag[k];
    x[k] = 0.0;
    r[k] = b;
    z[k] = zk;
    p1[k] = 0.0;
    rz += b * zk;
    bb += b * b;
  }
  block_sum2(rz, bb, part);
}

__global__ __launch_bounds__(kCgBlock) void k_cg_spmv(
    int nx, int ny, const double* __restrict__ diag, const double* __restrict__ cE,
    const double* __restrict__ cN, const double* __restrict__ z, double* __restrict__ P,
    double* __restrict__ q, double* __restrict__ part, const IterState* cs, const int* gate) {
  if ((gate && *gate) || cs->done) return;
  const long long n = (long long)nx * ny;
  const int it = cs->iter;
  const double beta = cs->beta;
  double* __restrict__ pk = P + (long long)(it & 1) * n;
  const double* __restrict__ pm = P + (long long)((it + 1) & 1) * n;
  double pq = 0.0;
  for (long long k = (long long)blockIdx.x * kCgBlock + threadIdx.x; k < n;
       k += (long long)gridDim.x * kCgBlock) {
    const int i = (int)(k % nx), j = (int)(k / nx);
    const double pc = z[k] + beta * pm[k];
    double a = 0.0;
    if (i + 1 < nx) a += cE[k] * (z[k + 1] + beta * pm[k + 1]);
    if (i > 0) a += cE[k - 1] * (z[k - 1] + beta * pm[k - 1]);
    if (j + 1 < ny) a += cN[k] * (z[k + nx] + beta * pm[k + nx]);
    if (j > 0) a += cN[k - nx] * (z[k - nx] + beta * pm[k - nx]);
    const double qk = diag[k] * pc - a;
    pk[k] = pc;
    q[k] = qk;
    pq += pc * qk;
  }
  block_sum2(pq, 0.0, part);
}

__global__ __launch_bounds__(kCgBlock) void k_cg_update(
    long long n, const double* __restrict__ diag, const double* __restrict__ P,
    const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ z, const double* __restrict__ part_pq, int n_part,
    double* __restrict__ part, const IterState* cs, const int* gate) {
  if ((gate && *gate) || cs->done) return;
  const double pq = sum_partials(part_pq, n_part, 0);
  const double alpha = cs->rz / pq;
  const double* __restrict__ pk = P + (long long)(cs->iter & 1) * n;
  double rz = 0.0, rr = 0.0;
  for (long long k = (long long)blockIdx.x * kCgBlock + threadIdx.x; k < n;
       k += (long long)gridDim.x * kCgBlock) {
    x[k] += alpha * pk[k];
    const double rk = r[k] - alpha * q[k];
    const double zk = rk / diag[k];
    r[k] = rk;
    z[k] = zk;
    rz += rk * zk;
    rr += rk * rk;
  }
  block_sum2(rz, rr, part);
}

__global__ __launch_bounds__(kCgBlock) void k_cg_residual(const double* part, int n_part,
                                                          IterState* cs, const int* gate,
                                                          double tol, int max_iter) {
  if ((gate && *gate) || cs->done) return;
  const double rz = sum_partials(part, n_part, 0);
  const double rr = sum_partials(part, n_part, 1);
  if (threadIdx.x == 0) {
    const double bb = cs->bb;
    cs->iter += 1;
    cs->dn2_prev = cs->dn2;
    cs->dn2 = rr;
    cs->nrm2 = bb;
    const int bad = !isfinite(rr) || !isfinite(rz);
    const int conv = !bad && rr <= tol * tol * bb;
    cs->bad = bad;
    cs->conv = conv;
    cs->done = bad || conv || cs->iter >= max_iter;
    cs->beta = cs->rz != 0.0 ? rz / cs->rz : 0.0;
    cs->rz = rz;
  }
}

// Small meshes (n <= kCgOneBlockMax): the whole solve in one workgroup of
// 1024 threads, the iterations separated by barriers instead of launches.
// Same iteration as above; the sums are formed per wave (shuffles in a fixed
// pattern) and then over the 16 wave sums in index order, by every thread,
// so every thread holds the same alpha, beta and decision.
constexpr int kCgOneBlock = 1024;
constexpr long long kCgOneBlockMax = 4096;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(kCgOneBlock) void k_cg_solve_one_block(
    int nx, int ny, const double* __restrict__ diag, const double* __restrict__ cE,
    const double* __restrict__ cN, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ z, double* __restrict__ P, double* __restrict__ q, IterState* cs,
    const int* gate, double tol, int max_iter) {
  if ((gate && *gate) || cs->done) return;
  __shared__ double s_a[kCgOneBlock / 64], s_b[kCgOneBlock / 64];
  const long long n = (long long)nx * ny;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  constexpr int nw = kCgOneBlock / 64;
  int it = cs->iter;
  double beta = cs->beta, rz = cs->rz;
  const double bb = cs->bb;
  double rr = 0.0;
  int done = 0, conv = 0, bad = 0;
  while (!done) {
    double* __restrict__ pk = P + (long long)(it & 1) * n;
    const double* __restrict__ pm = P + (long long)((it + 1) & 1) * n;
    double pq = 0.0;
    for (long long k = t; k < n; k += kCgOneBlock) {
      const int i = (int)(k % nx), j = (int)(k / nx);
      const double pc = z[k] + beta * pm[k];
      double a = 0.0;
      if (i + 1 < nx) a += cE[k] * (z[k + 1] + beta * pm[k + 1]);
      if (i > 0) a += cE[k - 1] * (z[k - 1] + beta * pm[k - 1]);
      if (j + 1 < ny) a += cN[k] * (z[k + nx] + beta * pm[k + nx]);
      if (j > 0) a += cN[k - nx] * (z[k - nx] + beta * pm[k - nx]);
      const double qk = diag[k] * pc - a;
      pk[k] = pc;
      q[k] = qk;
      pq += pc * qk;
    }
    pq = wave_sum(pq);
    if (lane == 0) s_a[wv] = pq;
    __syncthreads();
    pq = 0.0;
    for (int w = 0; w < nw; ++w) pq += s_a[w];
    const double alpha = rz / pq;
    double rzn = 0.0, rrn = 0.0;
    for (long long k = t; k < n; k += kCgOneBlock) {
      x[k] += alpha * pk[k];
      const double rk = r[k] - alpha * q[k];
      const double zk = rk / diag[k];
      r[k] = rk;
      z[k] = zk;
      rzn += rk * zk;
      rrn += rk * rk;
    }
    rzn = wave_sum(rzn);
    rrn = wave_sum(rrn);
    __syncthreads();  // every thread has read s_a; z of all cells is written
    if (lane == 0) {
      s_a[wv] = rzn;
      s_b[wv] = rrn;
    }
    __syncthreads();
    rzn = 0.0;
    rrn = 0.0;
    for (int w = 0; w < nw; ++w) {
      rzn += s_a[w];
      rrn += s_b[w];
    }
    __syncthreads();  // s_a, s_b are reused by the next iteration
    it += 1;
    rr = rrn;
    bad = !isfinite(rrn) || !isfinite(rzn);
    conv = !bad && rrn <= tol * tol * bb;
    done = bad || conv || it >= max_iter;
    beta = rz != 0.0 ? rzn / rz : 0.0;
    rz = rzn;
  }
  if (t == 0) {
    cs->iter = it;
    cs->dn2_prev = 0.0;
    cs->dn2 = rr;
    cs->nrm2 = bb;
    cs->bad = bad;
    cs->conv = conv;
    cs->done = 1;
    cs->beta = beta;
    cs->rz = rz;
  }
}

// phi_c nodal = the cell value at all four nodes.
__global__ void k_cg_to_nodal(long long n, const double* __restrict__ x,
                              double* __restrict__ phi_c, const int* halt) {
  if (*halt) return;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const double v = x[k];
    reinterpret_cast<double4*>(phi_c)[k] = make_double4(v, v, v, v);
  }
}

hipError_t launch_cg_start(const CgArgs& a, const double* sig_s, const double* phi_post,
                           int max_iter, const int* halt, hipStream_t s) {
  const long long n = (long long)a.nx * a.ny;
  hipLaunchKernelGGL(k_cg_start, dim3(a.n_part), dim3(kCgBlock), 0, s, n, sig_s, phi_post,
                     (const double*)a.diag, a.x, a.r, a.z, a.P + n, a.part_a, halt);
  hipLaunchKernelGGL(k_cg_start_state, dim3(1), dim3(kCgBlock), 0, s, (const double*)a.part_a,
                     a.n_part, a.cs, a.gate, max_iter, halt);
  return hipGetLastError();
}

hipError_t launch_dsa_start(const CgArgs& a, const double* sig_s, const double* dnode,
                            int max_iter, hipStream_t s) {
  const long long n = (long long)a.nx * a.ny;
  hipLaunchKernelGGL(k_dsa_start, dim3(a.n_part), dim3(kCgBlock), 0, s, n, sig_s, dnode,
                     (const double*)a.diag, a.x, a.r, a.z, a.P + n, a.part_a, a.gate);
  hipLaunchKernelGGL(k_cg_start_state, dim3(1), dim3(kCgBlock), 0, s, (const double*)a.part_a,
                     a.n_part, a.cs, a.gate, max_iter, (const int*)nullptr);
  return hipGetLastError();
}

bool cg_one_block(long long n) { return n <= kCgOneBlockMax; }

hipError_t launch_cg_solve_one_block(const CgArgs& a, double tol, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_solve_one_block, dim3(1), dim3(kCgOneBlock), 0, s, a.nx, a.ny,
                     (const double*)a.diag, (const double*)a.cE, (const double*)a.cN, a.x, a.r,
                     a.z, a.P, a.q, a.cs, a.gate, tol, max_iter);
  return hipGetLastError();
}

hipError_t launch_cg_iteration(const CgArgs& a, double tol, int max_iter, hipStream_t s) {
  const long long n = (long long)a.nx * a.ny;
  if (cg_one_block(n)) return launch_cg_solve_one_block(a, tol, max_iter, s);  // the whole rest
  hipLaunchKernelGGL(k_cg_spmv, dim3(a.n_part), dim3(kCgBlock), 0, s, a.nx, a.ny,
                     (const double*)a.diag, (const double*)a.cE, (const double*)a.cN,
                     (const double*)a.z, a.P, a.q, a.part_a, (const IterState*)a.cs, a.gate);
  hipLaunchKernelGGL(k_cg_update, dim3(a.n_part), dim3(kCgBlock), 0, s, n,
                     (const double*)a.diag, (const double*)a.P, (const double*)a.q, a.x, a.r,
                     a.z, (const double*)a.part_a, a.n_part, a.part_b, (const IterState*)a.cs,
                     a.gate);
  hipLaunchKernelGGL(k_cg_residual, dim3(1), dim3(kCgBlock), 0, s, (const double*)a.part_b,
                     a.n_part, a.cs, a.gate, tol, max_iter);
  return hipGetLastError();
}

hipError_t launch_cg_to_nodal(const CgArgs& a, double* phi_c, const int* halt, hipStream_t s) {
  const long long n = (long long)a.nx * a.ny;
  hipLaunchKernelGGL(k_cg_to_nodal, dim3(a.n_part), dim3(kCgBlock), 0, s, n,
                     (const double*)a.x, phi_c, halt);
  return hipGetLastError();
}

}  // namespace slh
