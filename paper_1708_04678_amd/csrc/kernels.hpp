// HIP kernels (gfx950) of one FE-LBM time step: D2Q9 populations g, h on a
// P1 triangle mesh (arXiv:1708.04678, Sec. II.A-D).
//
// Data layout (device, all structure-of-arrays):
//   populations  real [18][Np]   g_0..g_8 then h_0..h_8, Np = N rounded up to 64
//   node fields  C, mu, lap C in double; p, u_x, u_y in real
//   elements     tri/enbr int32 [3][E]; geometry double [7][E] = (A, grad N_0,
//                grad N_1, grad N_2) and a copy in real for the streaming gather
//   node->element gather list (CSR, packed element*4 + local vertex)
//   mass matrix  diag(m)^-1 M11 off-diagonal part in sliced-ELL form, slice
//                height 64 (one wavefront), column-major inside a slice
//
// Every node-indexed output is produced by exactly one thread that gathers its
// inputs (no scatter, no atomics): results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace felbm {

constexpr int Q = 9;
constexpr int NPOP = 18;

// D2Q9 velocity set and weights (textbook; the paper's 3-D runs use D3Q19)
__host__ __device__ constexpr int ex(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0); }
__host__ __device__ constexpr int ey(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0); }
__host__ __device__ constexpr double wq(int a) { return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : (a < 5 ? ((a + 1) % 4) + 1 : ((a - 3) % 4) + 5); }

// ----------------------------------------------------------------------------
// a1 + a6: moments, relaxation time, equilibria, BGK collision (eqn::collide)
// ----------------------------------------------------------------------------
// Reads the state psi_bar, writes the nodal fields and (COLLIDE) psi_hat in
// place; also writes per-block partials of the FP64 reductions of the state.
// In FP32 the composition is C = sum_a h_a + r with the FP64 remainder r
// (rC) carried between steps, see k_sweep.
template <typename real>
struct Conserve {
  static constexpr bool on = sizeof(real) == 4;
};

template <typename real, bool COLLIDE>
__global__ void __launch_bounds__(BLOCK) k_moments(real* __restrict__ pop, int N, int Np, StepParams P,
                                                  double* __restrict__ Cn, real* __restrict__ pn,
                                                  real* __restrict__ uxn, real* __restrict__ uyn,
                                                  const double* __restrict__ mass, const double* __restrict__ xy,
                                                  Band band, const double* __restrict__ rC,
                                                  double* __restrict__ partials) {
  const int blk = xcd_block();
  const int i = blk * BLOCK + threadIdx.x;
  double red[NRED] = {0, 0, 0, 0, 0, 0};
  if (i < N) {
    real g[Q], h[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      g[a] = pop[a * Np + i];
      h[a] = pop[(Q + a) * Np + i];
    }
    double C = 0.0;
    real p = 0, jx = 0, jy = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      C += (double)h[a];
      p += g[a];
      if (ex(a)) jx += ex(a) > 0 ? g[a] : -g[a];
      if (ey(a)) jy += ey(a) > 0 ? g[a] : -g[a];
    }
    if (Conserve<real>::on) C += rC[i];
    const real rho = (real)(C * P.rho_l + (1.0 - C) * P.rho_v);
    const real ux = (real)3.0 * jx / rho, uy = (real)3.0 * jy / rho;  // rho u = sum e g / c_s^2
    Cn[i] = C;
    pn[i] = p;
    uxn[i] = ux;
    uyn[i] = uy;
    if (COLLIDE) {
      const real tau = (real)(1.0 / (C * P.inv_tau_l + (1.0 - C) * P.inv_tau_v));
      const real om = (real)1 / (tau + (real)0.5);
      const real uu = ux * ux + uy * uy;
      const real Cr = (real)C;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const real eu = (real)ex(a) * ux + (real)ey(a) * uy;
        const real poly = eu + (real)1.5 * eu * eu - (real)0.5 * uu;   // c_s^2 (e.u/c_s^2 + ...)
        const real geq = (real)wq(a) * (p + rho * poly);
        const real heq = (real)wq(a) * Cr * ((real)1 + (real)3 * poly);
        pop[a * Np + i] = g[a] - om * (g[a] - geq);
        pop[(Q + a) * Np + i] = h[a] - om * (h[a] - heq);
      }
    }
    const double uu = (double)ux * ux + (double)uy * uy;
    const double rr = C * P.rho_l + (1.0 - C) * P.rho_v;
    red[0] = mass[i] * C;
    red[1] = rr * uu;
    red[2] = sqrt(uu);
    if (band.enabled) {
      double dx = xy[i] - band.xc;
      if (band.period > 0) dx -= band.period * rint(dx / band.period);
      const double dy = xy[N + i] - band.yc, d2 = dx * dx + dy * dy;
      if (d2 >= band.r_lo2 && d2 <= band.r_hi2) {
        red[3] = rr * uu;
        red[4] = 1.0;
      }
    }
    red[5] = (isfinite(C) && isfinite((double)p) && isfinite(uu)) ? 0.0 : 1.0;
    if (red[5] != 0.0) red[2] = 0.0;
  }
  block_reduce_store<NRED>(red, 2, partials, gridDim.x, blk);
}

// ----------------------------------------------------------------------------
// Residual of the mass-matrix solve (end of Sec. II.C) for a sampled step:
// with f = b/m and A = diag(m)^-1 M11, M11 x - b = m (A x - f), so in the
// norm ||v||^2 = sum_i v_i^2 / m_i the residual and the right-hand side are
// sum_i m_i (A x - f)_i^2 and sum_i m_i f_i^2 per population.  Block partials
// [2*18][nblk] in FP64, then one block forms max_a sqrt(res_a / rhs_a).
// Uses the sliced-ELL copy of A (present for every mesh).
// ----------------------------------------------------------------------------
constexpr int NRES = 2 * NPOP;

template <typename real>
__global__ void __launch_bounds__(BLOCK) k_residual(int N, int Np, const int* __restrict__ sell_ptr,
                                                   const int* __restrict__ sell_col, const real* __restrict__ sell_val,
                                                   const real* __restrict__ f, const real* __restrict__ x,
                                                   const double* __restrict__ mass, double* __restrict__ partials) {
  const int blk = xcd_block();
  const int i = blk * BLOCK + threadIdx.x;
  double v[NRES];
#pragma unroll
  for (int k = 0; k < NRES; ++k) v[k] = 0.0;
  if (i < N) {
    double acc[NPOP];
#pragma unroll
    for (int a = 0; a < NPOP; ++a) acc[a] = 0.5 * (double)x[a * Np + i];
    const int slice = i >> 6, lane = i & 63;
    const int base = sell_ptr[slice], width = (sell_ptr[slice + 1] - base) >> 6;
    for (int k = 0; k < width; ++k) {
      const int idx = base + (k << 6) + lane;
      const int j = sell_col[idx];
      const double aij = (double)sell_val[idx];
#pragma unroll
      for (int a = 0; a < NPOP; ++a) acc[a] += aij * (double)x[a * Np + j];
    }
    const double m = mass[i];
#pragma unroll
    for (int a = 0; a < NPOP; ++a) {
      const double fa = (double)f[a * Np + i], r = acc[a] - fa;
      v[a] = m * r * r;
      v[NPOP + a] = m * fa * fa;
    }
  }
  block_reduce_store<NRES>(v, -1, partials, gridDim.x, blk);
}

__global__ void __launch_bounds__(RBLOCK_RES) k_residual_final(const double* __restrict__ partials, int nblk,
                                                                double* __restrict__ out) {
  __shared__ double red[NRES][RBLOCK_RES / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < NRES; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RBLOCK_RES) s += partials[(size_t)k * nblk + b];
    s = wave_sum(s);
    if (lane == 0) red[k][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double worst = 0.0;
    for (int a = 0; a < NPOP; ++a) {
      double r = 0.0, fs = 0.0;
      for (int w = 0; w < RBLOCK_RES / 64; ++w) {
        r += red[a][w];
        fs += red[NPOP + a][w];
      }
      const double rel = fs > 0.0 ? sqrt(r / fs) : (r > 0.0 ? INFINITY : 0.0);
      worst = fmax(worst, rel);
    }
    *out = worst;
  }
}

// ----------------------------------------------------------------------------
// a2: element gradients of the P1 fields C (double) and p (real)
// ----------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_elem_grad(int E, const int* __restrict__ tri, const double* __restrict__ geo,
                                                    const double* __restrict__ Cn, const real* __restrict__ pn,
                                                    double* __restrict__ gC, real* __restrict__ gp) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= E) return;
  const int v0 = tri[e], v1 = tri[E + e], v2 = tri[2 * E + e];
  const double g0x = geo[E + e], g0y = geo[2 * E + e], g1x = geo[3 * E + e], g1y = geo[4 * E + e];
  const double g2x = geo[5 * E + e], g2y = geo[6 * E + e];
  const double c0 = Cn[v0], c1 = Cn[v1], c2 = Cn[v2];
  gC[e] = c0 * g0x + c1 * g1x + c2 * g2x;
  gC[E + e] = c0 * g0y + c1 * g1y + c2 * g2y;
  const real p0 = pn[v0], p1 = pn[v1], p2 = pn[v2];
  gp[e] = p0 * (real)g0x + p1 * (real)g1x + p2 * (real)g2x;
  gp[E + e] = p0 * (real)g0y + p1 * (real)g1y + p2 * (real)g2y;
}

// Outward flux through a wall edge from the wetting condition (eq. bc2, n
// into the fluid): -int (phi_c/kappa)(C - C^2) ds with C and phi_c/kappa
// linear on the edge, integrated exactly by Simpson's rule.
__device__ __forceinline__ double wall_flux(double Ca, double Cb, double ra, double rb, double len) {
  const double Cm = 0.5 * (Ca + Cb), rm = 0.5 * (ra + rb);
  return -len * (1.0 / 6.0) * (ra * (Ca - Ca * Ca) + 4.0 * rm * (Cm - Cm * Cm) + rb * (Cb - Cb * Cb));
}

// ----------------------------------------------------------------------------
// a3: nodal Laplacian of C over the vertex patch (eqn:lapl_int_mp) and the
// chemical potential mu = 2 beta C (C-1)(2C-1) - kappa lap C (eqn:mp_mu).
// The outer edge of patch element T opposite node k has |e| n_out =
// -2 A_T grad N_k; its gradient is the mean of the two adjacent element
// gradients; wall edges (opposite k, or incident to k) carry the wetting flux.
// Two passes: each element writes the flux through its three edges as seen
// from the opposite vertex (F[l][e]); each node sums the entries of its patch
// in its element-list order and adds the wall edges incident to it.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) k_edge_flux(int E, const int* __restrict__ tri, const int* __restrict__ enbr,
                                                    const double* __restrict__ geo, const double* __restrict__ gC,
                                                    const double* __restrict__ Cn, const double* __restrict__ bc,
                                                    double* __restrict__ F) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= E) return;
  const double A = geo[e], gCx = gC[e], gCy = gC[E + e];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double gx = geo[(1 + 2 * l) * E + e], gy = geo[(2 + 2 * l) * E + e];
    const int nb = enbr[l * E + e];
    double fl;
    if (nb >= 0) {
      const double Gx = 0.5 * (gCx + gC[nb]), Gy = 0.5 * (gCy + gC[E + nb]);
      fl = -2.0 * A * (gx * Gx + gy * Gy);
    } else {
      const int a = tri[((l + 1) % 3) * E + e], b = tri[((l + 2) % 3) * E + e];
      const double len = 2.0 * A * sqrt(gx * gx + gy * gy);
      fl = wall_flux(Cn[a], Cn[b], bc[a], bc[b], len);
    }
    F[l * E + e] = fl;
  }
}

__global__ void __launch_bounds__(BLOCK) k_lapC_mu(int N, int E, const int* __restrict__ n2e_ptr,
                                                  const int* __restrict__ n2e, const double* __restrict__ F,
                                                  const double* __restrict__ pvol, const double* __restrict__ Cn,
                                                  const double* __restrict__ bc, const int* __restrict__ wall_nbr,
                                                  const double* __restrict__ wall_len, StepParams P,
                                                  double* __restrict__ lapC, double* __restrict__ mu) {
  const int k = xcd_block() * BLOCK + threadIdx.x;
  if (k >= N) return;
  double flux = 0.0;
  const int beg = n2e_ptr[k], end = n2e_ptr[k + 1];
  for (int q = beg; q < end; ++q) {
    const int packed = n2e[q];
    flux += F[(packed & 3) * E + (packed >> 2)];
  }
  const double Ck = Cn[k];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int j = wall_nbr[w * N + k];
    if (j >= 0) flux += wall_flux(Ck, Cn[j], bc[k], bc[j], wall_len[w * N + k]);
  }
  const double L = flux / pvol[k];
  lapC[k] = L;
  mu[k] = 2.0 * P.beta * Ck * (Ck - 1.0) * (2.0 * Ck - 1.0) - P.kappa * L;
}

// ----------------------------------------------------------------------------
// a3 and a4 as precomputed linear operators (the time step's path).  The
// patch Laplacian with averaged outer-edge gradients (eqn:lapl_int_mp) is
// linear in the nodal C of the node's patch and of the elements across its
// outer edges; with the weights divided by the patch volume on the host,
//   lap C_k = sum_j w_kj (C_j - C_k) + sum_{wall edges e of the patch} F_BC(e) / |Omega_k|
// (difference form: sum_j w_kj = 0, so a constant field gives exactly 0).
// Rows in sliced-ELL form (slice height 64, column-major), padded with the
// node itself and weight 0; the wall edges of each patch in a short CSR list
// (a, b, |e| / |Omega_k|).  The element Laplacian of mu (Sec. II.D) is linear
// in mu at the element's vertices and at the three vertices across its edges:
//   lap mu_T = w1 (mu_1 - mu_0) + w2 (mu_2 - mu_0) + sum_l w_opp,l (mu_opp,l - mu_0),
// where an edge on a wall contributes nothing (eqn:bc1; its opposite slot
// points at vertex 0 with weight 0).  Values and arithmetic in FP64; the
// patch weights in the working precision (wreal), the element weights in
// FP64 (the FP32 composition transport relies on sum_T A_T lap mu_T = 0 to
// rounding, which FP32 weights would break by their rounding).
// ----------------------------------------------------------------------------
struct FieldOps {
  const int* lop_ptr;   // [Np/64 + 1] slice offsets
  const int* lop_col;   // [entries]
  const void* lop_w;    // [entries] wreal
  const int* wptr;      // [N+1] wall entries of each patch
  const int2* wab;      // [wall entries] edge end nodes
  const double* wlen;   // [wall entries] edge length / patch volume
  const int* eopp;      // [3][E] vertex across the edge opposite local vertex l (vertex 0 on a wall edge)
  const void* ew;       // [5][E] double in both precisions: A_T times these weights must cancel
                        // across each interior edge to rounding, which conserves mass
};

template <typename wreal, bool WRITE_LAPC>
__global__ void __launch_bounds__(BLOCK) k_lapC_mu_op(int N, FieldOps op, const double* __restrict__ Cn,
                                                     const double* __restrict__ bc, StepParams P,
                                                     double* __restrict__ lapC, double* __restrict__ mu) {
  const int k = xcd_block() * BLOCK + threadIdx.x;
  if (k >= N) return;
  const wreal* __restrict__ w = static_cast<const wreal*>(op.lop_w);
  const double Ck = Cn[k];
  const int slice = k >> 6, lane = k & 63;
  const int base = op.lop_ptr[slice], width = (op.lop_ptr[slice + 1] - base) >> 6;
  double acc = 0.0;
#pragma unroll 4
  for (int q = 0; q < width; ++q) {
    const int idx = base + (q << 6) + lane;
    acc += (double)w[idx] * (Cn[op.lop_col[idx]] - Ck);
  }
  for (int q = op.wptr[k]; q < op.wptr[k + 1]; ++q) {
    const int2 ab = op.wab[q];
    acc += wall_flux(Cn[ab.x], Cn[ab.y], bc[ab.x], bc[ab.y], op.wlen[q]);
  }
  if (WRITE_LAPC) lapC[k] = acc;
  mu[k] = 2.0 * P.beta * Ck * (Ck - 1.0) * (2.0 * Ck - 1.0) - P.kappa * acc;
}

__global__ void __launch_bounds__(BLOCK) k_lapmu_op(int E, const int* __restrict__ tri, FieldOps op,
                                                   const double* __restrict__ mu, double* __restrict__ lapmu) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= E) return;
  const double* __restrict__ w = static_cast<const double*>(op.ew);
  const double m0 = mu[tri[e]];
  const double d1 = mu[tri[E + e]] - m0, d2 = mu[tri[2 * E + e]] - m0;
  const double o0 = mu[op.eopp[e]] - m0, o1 = mu[op.eopp[E + e]] - m0, o2 = mu[op.eopp[2 * E + e]] - m0;
  lapmu[e] = w[e] * d1 + w[E + e] * d2 + w[2 * E + e] * o0 + w[3 * E + e] * o1 + w[4 * E + e] * o2;
}

// a4: element gradient of mu (P1) ...
__global__ void __launch_bounds__(BLOCK) k_elem_gradmu(int E, const int* __restrict__ tri,
                                                      const double* __restrict__ geo, const double* __restrict__ mu,
                                                      double* __restrict__ gmu) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= E) return;
  const double m0 = mu[tri[e]], m1 = mu[tri[E + e]], m2 = mu[tri[2 * E + e]];
  gmu[e] = m0 * geo[E + e] + m1 * geo[3 * E + e] + m2 * geo[5 * E + e];
  gmu[E + e] = m0 * geo[2 * E + e] + m1 * geo[4 * E + e] + m2 * geo[6 * E + e];
}

// ... and its element Laplacian (Sec. II.D): (1/A) sum over edges of
// |e| n . mean of the adjacent gradients, zero on wall edges (eqn:bc1);
// with |e| n = -2 A grad N_v this is -sum_v grad N_v . (g_T + g_T'(v)).
__global__ void __launch_bounds__(BLOCK) k_elem_lapmu(int E, const int* __restrict__ enbr,
                                                     const double* __restrict__ geo, const double* __restrict__ gmu,
                                                     double* __restrict__ lapmu) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= E) return;
  const double tx = gmu[e], ty = gmu[E + e];
  double acc = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int nb = enbr[l * E + e];
    if (nb >= 0) acc += geo[(1 + 2 * l) * E + e] * (tx + gmu[nb]) + geo[(2 + 2 * l) * E + e] * (ty + gmu[E + nb]);
  }
  lapmu[e] = -acc;
}

// ----------------------------------------------------------------------------
// a5 + a7: P0 element forces (eq:G, eq:H at barycentric values) fused into the
// node gather of the Galerkin streaming right-hand side (eq:galerkin_lbm):
//   b_{a,i} = sum_{T ni i} A_T q_{a,T} (dt/3 + dt^2/2 e_a . grad N_i|_T),
//   q_{a,T} = Phi_{a,T} - e_a . sum_{v in T} psi_hat_{a,v} grad N_v.
// Output f = b / m_i (the lumped solve, also the solver's initial guess).
// ----------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_rhs(int N, int Np, int E, const int* __restrict__ n2e_ptr,
                                              const int* __restrict__ n2e, const int* __restrict__ tri,
                                              const real* __restrict__ geor, const double* __restrict__ geo,
                                              const real* __restrict__ pn,
                                              const double* __restrict__ lapmu, const double* __restrict__ Cn,
                                              const real* __restrict__ uxn, const real* __restrict__ uyn,
                                              const double* __restrict__ mu, const real* __restrict__ pop,
                                              const double* __restrict__ mass, StepParams P, real* __restrict__ f,
                                              double* __restrict__ fC) {
  constexpr bool CONS = Conserve<real>::on;
  const int i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= N) return;
  real own[NPOP], b[NPOP];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) {
    own[a] = pop[a * Np + i];
    b[a] = 0;
  }
  double bC = 0.0;
  const real dt = (real)P.dt, c1 = dt / (real)3, c2 = (real)0.5 * dt * dt;
  const real drho_cs2 = (real)(CS2 * (P.rho_l - P.rho_v));
  const int beg = n2e_ptr[i], end = n2e_ptr[i + 1];
  for (int q = beg; q < end; ++q) {
    const int packed = n2e[q];
    const int e = packed >> 2, l = packed & 3;
    int v[3];
    v[0] = tri[e]; v[1] = tri[E + e]; v[2] = tri[2 * E + e];
    const real A = geor[e];
    real gx[3], gy[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      gx[t] = geor[(1 + 2 * t) * E + e];
      gy[t] = geor[(2 + 2 * t) * E + e];
    }
    // barycentric values of the P1 fields and the element gradients
    const double Cb = (Cn[v[0]] + Cn[v[1]] + Cn[v[2]]) * (1.0 / 3.0);
    const double mub = (mu[v[0]] + mu[v[1]] + mu[v[2]]) * (1.0 / 3.0);
    const real ux0 = uxn[v[0]], ux1 = uxn[v[1]], ux2 = uxn[v[2]];
    const real uy0 = uyn[v[0]], uy1 = uyn[v[1]], uy2 = uyn[v[2]];
    const real ubx = (ux0 + ux1 + ux2) / (real)3, uby = (uy0 + uy1 + uy2) / (real)3;
    const double rhobd = Cb * P.rho_l + (1.0 - Cb) * P.rho_v;
    const real rhob = (real)rhobd;
    // element gradients of the P1 fields C (FP64) and p (a2)
    const double Cv0 = Cn[v[0]], Cv1 = Cn[v[1]], Cv2 = Cn[v[2]];
    const double g0x = geo[E + e], g0y = geo[2 * E + e], g1x = geo[3 * E + e], g1y = geo[4 * E + e];
    const double g2x = geo[5 * E + e], g2y = geo[6 * E + e];
    const double gCx = Cv0 * g0x + Cv1 * g1x + Cv2 * g2x, gCy = Cv0 * g0y + Cv1 * g1y + Cv2 * g2y;
    const real pv0 = pn[v[0]], pv1 = pn[v[1]], pv2 = pn[v[2]];
    const real gpx = pv0 * (real)g0x + pv1 * (real)g1x + pv2 * (real)g2x;
    const real gpy = pv0 * (real)g0y + pv1 * (real)g1y + pv2 * (real)g2y;
    const real ax = drho_cs2 * (real)gCx, ay = drho_cs2 * (real)gCy;          // c_s^2 grad rho
    const real bx = (real)(mub * gCx), by = (real)(mub * gCy);                // mu grad C
    const real coef = (real)Cb / (rhob * (real)CS2);
    const real Xx = (real)gCx - coef * (gpx - bx), Xy = (real)gCy - coef * (gpy - by);
    const double lm = lapmu[e];
    const real d = (real)(P.mobility * lm);
    const real uA = ubx * ax + uby * ay, uB = ubx * bx + uby * by, uX = ubx * Xx + uby * Xy;
    const real uu = ubx * ubx + uby * uby;
    // post-collision populations of the two other vertices
    const int o1 = (l + 1) % 3, o2 = (l + 2) % 3;
    const int va = v[o1], vb = v[o2];
    real ha[Q], hb[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      ha[a] = pop[(Q + a) * Np + va];
      hb[a] = pop[(Q + a) * Np + vb];
    }
    const real gla = gx[o1], glb = gx[o2], hla = gy[o1], hlb = gy[o2];
    const real gxl = gx[l], gyl = gy[l];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const real exa = (real)ex(a), eya = (real)ey(a);
      const real eu = exa * ubx + eya * uby;
      const real G = (real)wq(a) * ((real)1 + (real)3 * eu + (real)4.5 * eu * eu - (real)1.5 * uu);
      const real Phig = (exa * ax + eya * ay - uA) * (G - (real)wq(a)) + (exa * bx + eya * by - uB) * G;
      const real Phih = (exa * Xx + eya * Xy - uX + d) * G;
      const real enl = exa * gxl + eya * gyl;
      const real ena = exa * gla + eya * hla, enb = exa * glb + eya * hlb;
      const real sg = own[a] * enl + pop[a * Np + va] * ena + pop[a * Np + vb] * enb;
      const real sh = own[Q + a] * enl + ha[a] * ena + hb[a] * enb;
      const real wgt = A * (c1 + c2 * enl);
      b[a] += wgt * (Phig - sg);
      b[Q + a] += wgt * (Phih - sh);
    }
    if (CONS) {
      // zeroth h-moment of this element's contribution in FP64 from the moment
      // identities of Gamma (sum Gamma = 1, sum e Gamma = u, sum e e Gamma =
      // c_s^2 I + u u): sum_a q_a = M lap mu - div J, sum_a e_a q_a =
      // c_s^2 X + M lap mu u - div Pi, with J = sum e h_hat, Pi = sum e e h_hat.
      // Evaluated in the element's fixed vertex order so that the three
      // vertices' shares are bitwise identical and telescope.
      double Jx[3], Jy[3], Pxx[3], Pxy[3], Pyy[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) { Jx[t] = Jy[t] = Pxx[t] = Pxy[t] = Pyy[t] = 0.0; }
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const double hv[3] = {(double)(l == 0 ? own[Q + a] : (o1 == 0 ? ha[a] : hb[a])),
                              (double)(l == 1 ? own[Q + a] : (o1 == 1 ? ha[a] : hb[a])),
                              (double)(l == 2 ? own[Q + a] : (o1 == 2 ? ha[a] : hb[a]))};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          if (ex(a)) Jx[t] += ex(a) * hv[t];
          if (ey(a)) Jy[t] += ey(a) * hv[t];
          if (ex(a)) Pxx[t] += hv[t];
          if (ex(a) && ey(a)) Pxy[t] += ex(a) * ey(a) * hv[t];
          if (ey(a)) Pyy[t] += hv[t];
        }
      }
      const double Ad = geo[e];
      double gxd[3], gyd[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        gxd[t] = geo[(1 + 2 * t) * E + e];
        gyd[t] = geo[(2 + 2 * t) * E + e];
      }
      double divJ = 0.0, dPx = 0.0, dPy = 0.0;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        divJ += gxd[t] * Jx[t] + gyd[t] * Jy[t];
        dPx += gxd[t] * Pxx[t] + gyd[t] * Pxy[t];
        dPy += gxd[t] * Pxy[t] + gyd[t] * Pyy[t];
      }
      const double uxd = ((double)ux0 + (double)ux1 + (double)ux2) * (1.0 / 3.0);
      const double uyd = ((double)uy0 + (double)uy1 + (double)uy2) * (1.0 / 3.0);
      const double cf = Cb / (rhobd * CS2);
      const double Xdx = gCx - cf * ((double)gpx - mub * gCx), Xdy = gCy - cf * ((double)gpy - mub * gCy);
      const double Ml = P.mobility * lm;
      const double s0 = Ml - divJ;
      const double s1x = CS2 * Xdx + Ml * uxd - dPx, s1y = CS2 * Xdy + Ml * uyd - dPy;
      bC += Ad * (P.dt * (1.0 / 3.0) * s0 + 0.5 * P.dt * P.dt * (gxd[l] * s1x + gyd[l] * s1y));
    }
  }
  const real inv_m = (real)(1.0 / mass[i]);
#pragma unroll
  for (int a = 0; a < NPOP; ++a) f[a * Np + i] = b[a] * inv_m;
  if (CONS) fC[i] = bC / mass[i];
}

// ----------------------------------------------------------------------------
// Nodal (P1) forces, the comparison scheme of the parasitic-current table
// (Sec. III.A), which the paper names but does not spell out.  Reading: the
// same eq:G / eq:H, evaluated at the nodes with nodal values of the fields
// and with nodal gradients (area-weighted means of the element gradients over
// the vertex patch), nodal lap mu from the vertex-patch operator of
// eqn:lapl_int_mp with zero flux through wall edges (eqn:bc1); the force then
// enters the streaming step as a P1 field: + dt int phi_i F
// + dt^2/2 int (e . grad phi_i) F.  FP64.
// ----------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_node_forces(int N, int Np, int E, const int* __restrict__ n2e_ptr,
                                                      const int* __restrict__ n2e, const int* __restrict__ enbr,
                                                      const double* __restrict__ geo, const double* __restrict__ pvol,
                                                      const double* __restrict__ gC, const real* __restrict__ gp,
                                                      const double* __restrict__ gmu, const double* __restrict__ Cn,
                                                      const real* __restrict__ uxn, const real* __restrict__ uyn,
                                                      const double* __restrict__ mu, StepParams P,
                                                      real* __restrict__ Fn) {
  const int i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= N) return;
  double sCx = 0.0, sCy = 0.0, spx = 0.0, spy = 0.0, flux = 0.0;
  for (int q = n2e_ptr[i]; q < n2e_ptr[i + 1]; ++q) {
    const int packed = n2e[q];
    const int e = packed >> 2, l = packed & 3;
    const double A = geo[e];
    sCx += A * gC[e];
    sCy += A * gC[E + e];
    spx += A * (double)gp[e];
    spy += A * (double)gp[E + e];
    const int nb = enbr[l * E + e];
    if (nb >= 0) {
      const double Gx = 0.5 * (gmu[e] + gmu[nb]), Gy = 0.5 * (gmu[E + e] + gmu[E + nb]);
      flux += -2.0 * A * (geo[(1 + 2 * l) * E + e] * Gx + geo[(2 + 2 * l) * E + e] * Gy);
    }
  }
  const double vol = pvol[i];
  const double gCx = sCx / vol, gCy = sCy / vol, gpx = spx / vol, gpy = spy / vol, lm = flux / vol;
  const double C = Cn[i], m = mu[i];
  const double rho = C * P.rho_l + (1.0 - C) * P.rho_v;
  const double ux = (double)uxn[i], uy = (double)uyn[i];
  const double drho = P.rho_l - P.rho_v;
  const double ax = CS2 * drho * gCx, ay = CS2 * drho * gCy;  // c_s^2 grad rho
  const double bx = m * gCx, by = m * gCy;                    // mu grad C
  const double cf = C / (rho * CS2);
  const double Xx = gCx - cf * (gpx - bx), Xy = gCy - cf * (gpy - by);
  const double d = P.mobility * lm;
  const double uu = ux * ux + uy * uy;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy;
    const double G = wq(a) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    const double Fg = ((ex(a) - ux) * ax + (ey(a) - uy) * ay) * (G - wq(a)) + ((ex(a) - ux) * bx + (ey(a) - uy) * by) * G;
    const double Fh = ((ex(a) - ux) * Xx + (ey(a) - uy) * Xy + d) * G;
    Fn[a * Np + i] = (real)Fg;
    Fn[(Q + a) * Np + i] = (real)Fh;
  }
}

// Galerkin right-hand side with the P1 force: per incident element,
//   b_{a,i} += -A (dt/3 + dt^2/2 e_a . grad N_i) e_a . sum_v psi_hat_{a,v} grad N_v
//            + dt A/12 (F_{a,i} + sum_v F_{a,v}) + dt^2/2 (e_a . grad N_i) A/3 sum_v F_{a,v}
// (the consistent P1 mass and 1/2 int (e . grad phi_i) phi_j); f = b / m.
template <typename real, bool FORCE>
__global__ void __launch_bounds__(BLOCK) k_rhs_nodal(int N, int Np, int E, const int* __restrict__ n2e_ptr,
                                                    const int* __restrict__ n2e, const int* __restrict__ tri,
                                                    const double* __restrict__ geo, const real* __restrict__ Fn,
                                                    const real* __restrict__ pop, const double* __restrict__ mass,
                                                    StepParams P, real* __restrict__ f) {
  const int i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= N) return;
  real b[NPOP];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) b[a] = (real)0;
  const real dt = (real)P.dt, c1 = dt / (real)3, c2 = (real)0.5 * dt * dt;
  for (int q = n2e_ptr[i]; q < n2e_ptr[i + 1]; ++q) {
    const int packed = n2e[q];
    const int e = packed >> 2, l = packed & 3;
    const int v0 = tri[e], v1 = tri[E + e], v2 = tri[2 * E + e];
    const real A = (real)geo[e];
    real gx[3], gy[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      gx[t] = (real)geo[(1 + 2 * t) * E + e];
      gy[t] = (real)geo[(2 + 2 * t) * E + e];
    }
    const real gxl = l == 0 ? gx[0] : (l == 1 ? gx[1] : gx[2]);
    const real gyl = l == 0 ? gy[0] : (l == 1 ? gy[1] : gy[2]);
#pragma unroll
    for (int a = 0; a < NPOP; ++a) {
      const int d = a < Q ? a : a - Q;
      const real exa = (real)ex(d), eya = (real)ey(d);
      const real s = pop[a * Np + v0] * (exa * gx[0] + eya * gy[0]) + pop[a * Np + v1] * (exa * gx[1] + eya * gy[1]) +
                     pop[a * Np + v2] * (exa * gx[2] + eya * gy[2]);
      const real enl = exa * gxl + eya * gyl;
      b[a] += -A * (c1 + c2 * enl) * s;
      if (FORCE) {
        const real F0 = Fn[a * Np + v0], F1 = Fn[a * Np + v1], F2 = Fn[a * Np + v2];
        const real Fi = Fn[a * Np + i];
        const real fsum = F0 + F1 + F2;
        b[a] += dt * (A / (real)12) * (Fi + fsum) + c2 * enl * (A / (real)3) * fsum;
      }
    }
  }
  const real inv_m = (real)(1.0 / mass[i]);
#pragma unroll
  for (int a = 0; a < NPOP; ++a) f[a * Np + i] = b[a] * inv_m;
}

// ----------------------------------------------------------------------------
// Nodal forces integrated in the collision step, the comparison scheme of the
// authors' earlier work (parasitic-current table, Sec. III.A; Sec. II.C names
// it).  The trapezoid rule of eqn::integrated is applied to the force as to
// the BGK term, with psi_bar = psi + dt/2 (Omega - F), so that
//   psi_hat = psi_bar - (psi_bar - psi_eq + dt/2 F)/(tau + 1/2) + dt F
// and the streaming carries no force.  The moments of psi_bar then carry half
// the force's: rho u = sum e g / c_s^2 + dt/2 mu grad C and
// p = sum g + dt/2 c_s^2 u . grad rho; the fields use C = sum h, the h
// equilibrium C* = C + dt/2 M lap mu (so sum h_hat = sum h_bar + dt M lap mu).
// Nodal gradients are area-weighted patch means of the element gradients,
// nodal lap mu the patch operator of eqn:lapl_int_mp with zero wall flux; wall
// nodes are at rest: u = 0, F_g = 0, F_h = M lap mu w.  FP64.
// ----------------------------------------------------------------------------
template <typename real, bool CORRECT>
__global__ void __launch_bounds__(BLOCK) k_nc_fields(int N, int E, const int* __restrict__ n2e_ptr, const int* __restrict__ n2e,
                                                    const int* __restrict__ enbr, const double* __restrict__ geo,
                                                    const double* __restrict__ pvol, const double* __restrict__ gC,
                                                    const double* __restrict__ gmu, const double* __restrict__ Cn,
                                                    const double* __restrict__ mu, const uint8_t* __restrict__ is_wall,
                                                    StepParams P, real* __restrict__ pn, real* __restrict__ uxn,
                                                    real* __restrict__ uyn, double* __restrict__ lapmu_n,
                                                    const double* __restrict__ mass, const double* __restrict__ xy,
                                                    Band band, double* __restrict__ partials) {
  const int blk = xcd_block();
  const int i = blk * BLOCK + threadIdx.x;
  double red[NRED] = {0, 0, 0, 0, 0, 0};
  if (i < N) {
    double sCx = 0.0, sCy = 0.0, flux = 0.0;
    for (int q = n2e_ptr[i]; q < n2e_ptr[i + 1]; ++q) {
      const int packed = n2e[q];
      const int e = packed >> 2, l = packed & 3;
      const double A = geo[e];
      sCx += A * gC[e];
      sCy += A * gC[E + e];
      const int nb = enbr[l * E + e];
      if (nb >= 0) {
        const double Gx = 0.5 * (gmu[e] + gmu[nb]), Gy = 0.5 * (gmu[E + e] + gmu[E + nb]);
        flux += -2.0 * A * (geo[(1 + 2 * l) * E + e] * Gx + geo[(2 + 2 * l) * E + e] * Gy);
      }
    }
    const double vol = pvol[i];
    const double gCx = sCx / vol, gCy = sCy / vol;
    lapmu_n[i] = flux / vol;
    const double C = Cn[i];
    const double rho = C * P.rho_l + (1.0 - C) * P.rho_v;
    double ux = (double)uxn[i], uy = (double)uyn[i], p = (double)pn[i];
    if (CORRECT) {
      if (is_wall[i]) {
        ux = 0.0;
        uy = 0.0;
      } else {
        const double s = 0.5 * P.dt * mu[i] / rho;
        ux += s * gCx;
        uy += s * gCy;
      }
      p += 0.5 * P.dt * CS2 * (P.rho_l - P.rho_v) * (ux * gCx + uy * gCy);
      uxn[i] = (real)ux;
      uyn[i] = (real)uy;
      pn[i] = (real)p;
    }
    const double uu = ux * ux + uy * uy;
    red[0] = mass[i] * C;
    red[1] = rho * uu;
    red[2] = sqrt(uu);
    if (band.enabled) {
      double dx = xy[i] - band.xc;
      if (band.period > 0) dx -= band.period * rint(dx / band.period);
      const double dy = xy[N + i] - band.yc, d2 = dx * dx + dy * dy;
      if (d2 >= band.r_lo2 && d2 <= band.r_hi2) {
        red[3] = rho * uu;
        red[4] = 1.0;
      }
    }
    red[5] = (isfinite(C) && isfinite(p) && isfinite(uu)) ? 0.0 : 1.0;
    if (red[5] != 0.0) red[2] = 0.0;
  }
  block_reduce_store<NRED>(red, 2, partials, gridDim.x, blk);
}

// INIT = false: the collision with the force.  INIT = true: the initial state
// psi_bar^0 = psi_eq - dt/2 F (populations at equilibrium on entry); for h only
// the part of F_h with zero sum, so that sum h_bar^0 = C.
template <typename real, bool INIT>
__global__ void __launch_bounds__(BLOCK) k_nc_collide(int N, int Np, int E, const int* __restrict__ n2e_ptr,
                                                     const int* __restrict__ n2e, const double* __restrict__ geo,
                                                     const double* __restrict__ pvol, const double* __restrict__ gC,
                                                     const real* __restrict__ gp, const double* __restrict__ Cn,
                                                     const real* __restrict__ pn, const real* __restrict__ uxn,
                                                     const real* __restrict__ uyn, const double* __restrict__ mu,
                                                     const double* __restrict__ lapmu_n,
                                                     const uint8_t* __restrict__ is_wall, StepParams P,
                                                     real* __restrict__ pop) {
  const int i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= N) return;
  double sCx = 0.0, sCy = 0.0, spx = 0.0, spy = 0.0;
  for (int q = n2e_ptr[i]; q < n2e_ptr[i + 1]; ++q) {
    const int e = n2e[q] >> 2;
    const double A = geo[e];
    sCx += A * gC[e];
    sCy += A * gC[E + e];
    spx += A * (double)gp[e];
    spy += A * (double)gp[E + e];
  }
  const double vol = pvol[i];
  const double gCx = sCx / vol, gCy = sCy / vol, gpx = spx / vol, gpy = spy / vol;
  const double C = Cn[i], m = mu[i], lm = lapmu_n[i], p = (double)pn[i];
  const double ux = (double)uxn[i], uy = (double)uyn[i];
  const double rho = C * P.rho_l + (1.0 - C) * P.rho_v;
  const double drho = P.rho_l - P.rho_v;
  const double ax = CS2 * drho * gCx, ay = CS2 * drho * gCy;  // c_s^2 grad rho
  const double bx = m * gCx, by = m * gCy;                    // mu grad C
  const double cf = C / (rho * CS2);
  const double Xx = gCx - cf * (gpx - bx), Xy = gCy - cf * (gpy - by);
  const double d = P.mobility * lm;
  const double uu = ux * ux + uy * uy;
  const bool wall = is_wall[i] != 0;
  const double tau = 1.0 / (C * P.inv_tau_l + (1.0 - C) * P.inv_tau_v);
  const double om = 1.0 / (tau + 0.5);
  const double Cs = C + 0.5 * P.dt * d;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy;
    const double G = wq(a) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    double Fg, Fh, odd;
    if (wall) {
      Fg = 0.0;
      Fh = d * wq(a);
      odd = 0.0;
    } else {
      Fg = ((ex(a) - ux) * ax + (ey(a) - uy) * ay) * (G - wq(a)) + ((ex(a) - ux) * bx + (ey(a) - uy) * by) * G;
      odd = ((ex(a) - ux) * Xx + (ey(a) - uy) * Xy) * G;
      Fh = odd + d * G;
    }
    const double g = (double)pop[a * Np + i], h = (double)pop[(Q + a) * Np + i];
    if (INIT) {
      pop[a * Np + i] = (real)(g - 0.5 * P.dt * Fg);
      pop[(Q + a) * Np + i] = (real)(h - 0.5 * P.dt * odd);
    } else {
      const double poly = eu + 1.5 * eu * eu - 0.5 * uu;
      const double geq = wq(a) * (p + rho * poly);
      const double heq = wq(a) * Cs * (1.0 + 3.0 * poly);
      pop[a * Np + i] = (real)(g - om * (g - geq + 0.5 * P.dt * Fg) + P.dt * Fg);
      pop[(Q + a) * Np + i] = (real)(h - om * (h - heq + 0.5 * P.dt * Fh) + P.dt * Fh);
    }
  }
}

// ----------------------------------------------------------------------------
// Tiles of 256 consecutive (internal-order) nodes, their halo lists and LDS
// slots, shared by the LDS-staged right-hand side and solve sweeps.
// ----------------------------------------------------------------------------
constexpr int TILE = BLOCK;
constexpr int MAXW = 12;
// compile-time LDS strides (so that population offsets are instruction
// immediates): halo of a tile <= 128 nodes
constexpr int HALO_MAX = 128;
constexpr int SLOTS1 = TILE + HALO_MAX;  // tile + halo

struct TileArgs {
  const int* tile_off;   // [ntiles+1] entry offsets
  const uint16_t* slot;  // [entries]
  const int* halo_off;   // [ntiles+1]
  const int* halo;       // halo node ids
  int ntiles, slots;     // slots = 256 + largest halo
};

typedef __attribute__((address_space(3))) void lds_void_t;

// each active lane's 16 (4) bytes at src land at lds_wave_base + lane * 16 (4)
__device__ __forceinline__ void lds_dma16(const void* src, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(src, (lds_void_t*)lds_wave_base, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma4(const void* src, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(src, (lds_void_t*)lds_wave_base, 4, 0, 0);
}

// streamed accesses (read or written once per launch, no reuse inside it):
// nontemporal when NT, ordinary otherwise
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ----------------------------------------------------------------------------
// The same right-hand side with the vertex data of a 256-node tile and its
// halo staged in LDS: post-collision populations (tile by 16-byte LDS DMA; FP32
// halo by 4-byte DMA gathers, FP64 halo through registers), the nodal fields
// C, mu, u by ordinary loads.  Thread = node; its incident elements are
// listed per tile column-major (entry k of lane l at ent_off[t] + k*256 + l):
// x = element * 4 + local vertex (-1 = padding), y = LDS slots of the
// element's vertices 0, 1, 2 (9 bits each).  Element data (geometry as one
// FP64 record, lap mu) is read from global memory, the geometry rounded to the
// working precision where the arithmetic is; the element gradients of C and
// p come from the staged vertex values.  Every element sum runs over the
// vertices in the order 0, 1, 2, so the three vertices of an element form the
// same streaming derivative; only the test-function weight is the gathering
// vertex's own.  FP32 only: the FP64 zeroth h-moment uses
// div J = sum_a s_a, div Pi = sum_a e_a s_a with
// s_a = sum_v (e_a . grad N_v) h_hat_{a,v}, as in k_rhs.  The FP32 form is held
// to 128 VGPRs, so that four workgroups per CU (the LDS limit) are resident.
// ----------------------------------------------------------------------------
template <typename real>
constexpr unsigned rhs_lds_bytes() {
  return NPOP * SLOTS1 * sizeof(real) + SLOTS1 * (8 + 8 + 3 * sizeof(real));
}
struct RhsTile {
  const int* ent_off;   // [ntiles+1]
  const int2* ent;      // [entries]
  const double* gaos;   // [E][4] FP64 element geometry {dN1/dx, dN1/dy, dN2/dx, dN2/dy}
  const double* lapmu;  // [E]
};

template <typename real>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? 4 : 1))) k_rhs_lds(int N, int Np, int E, TileArgs ta, RhsTile rt,
                                                  const double* __restrict__ Cn, const real* __restrict__ pn,
                                                  const real* __restrict__ uxn,
                                                  const real* __restrict__ uyn, const double* __restrict__ mu,
                                                  const real* __restrict__ pop, const double* __restrict__ mass,
                                                  StepParams P, real* __restrict__ f, double* __restrict__ fC) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int S = SLOTS1;
  constexpr bool CONS = Conserve<real>::on;
  real* ps = reinterpret_cast<real*>(smem);
  double* Cs = reinterpret_cast<double*>(smem + NPOP * S * sizeof(real));
  double* mus = Cs + S;
  real* uxs = reinterpret_cast<real*>(mus + S);
  real* uys = uxs + S;
  real* pps = uys + S;
  const int t = xcd_block();
  if (t >= ta.ntiles) return;  // block-uniform
  const int lane = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(lane >> 6);
  const int l64 = lane & 63;
  const int base = t * TILE;
  const int i = base + lane;
  const bool valid = i < N;
  const int h0 = ta.halo_off[t], nh = ta.halo_off[t + 1] - h0;
  constexpr int PER = 16 / sizeof(real);  // values per lane and 16-byte load
#pragma unroll
  for (int c = 0; c < TILE / (64 * PER); ++c)
    if (base + c * 64 * PER + PER * l64 < Np)
      for (int a = wave; a < NPOP; a += 4)
        lds_dma16(pop + a * Np + base + c * 64 * PER + PER * l64, ps + a * S + c * 64 * PER);
  const int hid0 = l64 < nh ? ta.halo[h0 + l64] : 0;
  const int hid1 = 64 + l64 < nh ? ta.halo[h0 + 64 + l64] : 0;
  for (int a = wave; a < NPOP; a += 4) {
    if constexpr (sizeof(real) == 4) {
      if (l64 < nh) lds_dma4(pop + a * Np + hid0, ps + a * S + TILE);
      if (64 + l64 < nh) lds_dma4(pop + a * Np + hid1, ps + a * S + TILE + 64);
    } else {
      // 8-byte halo values go through registers (LDS DMA moves at most 4 bytes per gathered lane)
      if (l64 < nh) ps[a * S + TILE + l64] = pop[a * Np + hid0];
      if (64 + l64 < nh) ps[a * S + TILE + 64 + l64] = pop[a * Np + hid1];
    }
  }
  if (valid) {
    Cs[lane] = Cn[i];
    mus[lane] = mu[i];
    uxs[lane] = uxn[i];
    uys[lane] = uyn[i];
    pps[lane] = pn[i];
  }
  if (lane < nh) {
    const int j = ta.halo[h0 + lane];
    Cs[TILE + lane] = Cn[j];
    mus[TILE + lane] = mu[j];
    uxs[TILE + lane] = uxn[j];
    uys[TILE + lane] = uyn[j];
    pps[TILE + lane] = pn[j];
  }
  const double mi = valid ? mass[i] : 1.0;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's LDS DMA has landed
  __syncthreads();
  if (!valid) return;
  real b[NPOP];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) b[a] = (real)0;
  double bC = 0.0;
  const real dt = (real)P.dt, c1 = dt / (real)3, c2 = (real)0.5 * dt * dt;
  const real drho_cs2 = (real)(CS2 * (P.rho_l - P.rho_v));
  const int e0 = rt.ent_off[t], width = (rt.ent_off[t + 1] - e0) / TILE;
  // the next entry is loaded one iteration ahead, so that only the element
  // data wait on memory inside the loop
  int2 en_next = width > 0 ? rt.ent[e0 + lane] : int2{-1, 0};
  for (int k = 0; k < width; ++k) {
    const int2 en = en_next;
    if (k + 1 < width) en_next = rt.ent[e0 + (k + 1) * TILE + lane];
    if (en.x < 0) continue;
    const int e = en.x >> 2, l = en.x & 3;
    const int s0 = en.y & 511, s1 = (en.y >> 9) & 511, s2 = (en.y >> 18) & 511;
    // the element's geometry as one 32-byte record {grad N1, grad N2}; grad N0 =
    // -(grad N1 + grad N2) and A = 1 / (2 det[grad N1; grad N2]) are recomputed
    // (the same values at all three vertices of the element)
    const double2* g2 = reinterpret_cast<const double2*>(rt.gaos) + 2 * (size_t)e;
    const double2 ga = g2[0], gb = g2[1];
    const double Ad = 0.5 / (ga.x * gb.y - ga.y * gb.x);
    const double gxd[3] = {-(ga.x + gb.x), ga.x, gb.x}, gyd[3] = {-(ga.y + gb.y), ga.y, gb.y};
    real gxf[3], gyf[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      gxf[v] = (real)gxd[v];
      gyf[v] = (real)gyd[v];
    }
    const real A = (real)Ad;
    // the gathering vertex's shape-function gradient (test function of the row)
    const real gxl = l == 0 ? gxf[0] : (l == 1 ? gxf[1] : gxf[2]);
    const real gyl = l == 0 ? gyf[0] : (l == 1 ? gyf[1] : gyf[2]);
    // barycentric values of the P1 fields and the element gradients
    const double Cb = (Cs[s0] + Cs[s1] + Cs[s2]) * (1.0 / 3.0);  // barycentric values
    const double mub = (mus[s0] + mus[s1] + mus[s2]) * (1.0 / 3.0);
    const real ux0 = uxs[s0], ux1 = uxs[s1], ux2 = uxs[s2];
    const real uy0 = uys[s0], uy1 = uys[s1], uy2 = uys[s2];
    const real ubx = (ux0 + ux1 + ux2) / (real)3, uby = (uy0 + uy1 + uy2) / (real)3;
    const double rhobd = Cb * P.rho_l + (1.0 - Cb) * P.rho_v;
    const real rhob = (real)rhobd;
    // element gradients of the P1 fields C (FP64) and p (a2), from the staged vertex values
    const double Cv0 = Cs[s0], Cv1 = Cs[s1], Cv2 = Cs[s2];
    const double gCx = Cv0 * gxd[0] + Cv1 * gxd[1] + Cv2 * gxd[2], gCy = Cv0 * gyd[0] + Cv1 * gyd[1] + Cv2 * gyd[2];
    const real pv0 = pps[s0], pv1 = pps[s1], pv2 = pps[s2];
    const real gpx = pv0 * gxf[0] + pv1 * gxf[1] + pv2 * gxf[2], gpy = pv0 * gyf[0] + pv1 * gyf[1] + pv2 * gyf[2];
    const real ax = drho_cs2 * (real)gCx, ay = drho_cs2 * (real)gCy;  // c_s^2 grad rho
    const real bx = (real)(mub * gCx), by = (real)(mub * gCy);        // mu grad C
    const real coef = (real)Cb / (rhob * (real)CS2);
    const real Xx = (real)gCx - coef * (gpx - bx), Xy = (real)gCy - coef * (gpy - by);
    const double lm = rt.lapmu[e];
    const real d = (real)(P.mobility * lm);
    const real uA = ubx * ax + uby * ay, uB = ubx * bx + uby * by, uX = ubx * Xx + uby * Xy;
    const real uu = ubx * ubx + uby * uby;
    // FP32 only: the parts of the FP64 composition moment that do not depend on
    // h, formed before the direction loop so that only six doubles stay live
    // through it: bC += cw0 (M lap mu - div J) + cwl . (s1 - div Pi), with
    // s1 = c_s^2 X + M lap mu u and cw0 = A dt / 3, cwl = A dt^2 / 2 grad N_l
    double cw0 = 0.0, cwx = 0.0, cwy = 0.0, Ml = 0.0, s1x = 0.0, s1y = 0.0;
    if (CONS) {
      const double uxd = ((double)ux0 + (double)ux1 + (double)ux2) * (1.0 / 3.0);
      const double uyd = ((double)uy0 + (double)uy1 + (double)uy2) * (1.0 / 3.0);
      const double cf = Cb / (rhobd * CS2);
      const double Xdx = gCx - cf * ((double)gpx - mub * gCx), Xdy = gCy - cf * ((double)gpy - mub * gCy);
      Ml = P.mobility * lm;
      s1x = CS2 * Xdx + Ml * uxd;
      s1y = CS2 * Xdy + Ml * uyd;
      const double gxl_d = l == 0 ? gxd[0] : (l == 1 ? gxd[1] : gxd[2]);
      const double gyl_d = l == 0 ? gyd[0] : (l == 1 ? gyd[1] : gyd[2]);
      const double c2d = Ad * (0.5 * P.dt * P.dt);
      cw0 = Ad * (P.dt * (1.0 / 3.0));
      cwx = c2d * gxl_d;
      cwy = c2d * gyl_d;
    }
    double divJ = 0.0, dPx = 0.0, dPy = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const real exa = (real)ex(a), eya = (real)ey(a);
      const real eu = exa * ubx + eya * uby;
      const real G = (real)wq(a) * ((real)1 + (real)3 * eu + (real)4.5 * eu * eu - (real)1.5 * uu);
      const real Phig = (exa * ax + eya * ay - uA) * (G - (real)wq(a)) + (exa * bx + eya * by - uB) * G;
      const real Phih = (exa * Xx + eya * Xy - uX + d) * G;
      // the element's streaming derivative e_a . grad psi_a over its vertices in
      // the order 0, 1, 2, the same at each of the three gathering vertices
      const real en0 = exa * gxf[0] + eya * gyf[0], en1 = exa * gxf[1] + eya * gyf[1];
      const real en2 = exa * gxf[2] + eya * gyf[2], enl = exa * gxl + eya * gyl;
      const real h0 = ps[(Q + a) * S + s0], h1 = ps[(Q + a) * S + s1], h2 = ps[(Q + a) * S + s2];
      const real sg = ps[a * S + s0] * en0 + ps[a * S + s1] * en1 + ps[a * S + s2] * en2;
      const real sh = h0 * en0 + h1 * en1 + h2 * en2;
      const real wgt = A * (c1 + c2 * enl);
      b[a] += wgt * (Phig - sg);
      b[Q + a] += wgt * (Phih - sh);
      if (CONS && a != 0) {
        const double sa_d = (ex(a) * gxd[0] + ey(a) * gyd[0]) * (double)h0 +
                            (ex(a) * gxd[1] + ey(a) * gyd[1]) * (double)h1 +
                            (ex(a) * gxd[2] + ey(a) * gyd[2]) * (double)h2;
        divJ += sa_d;
        if (ex(a)) dPx += ex(a) * sa_d;
        if (ey(a)) dPy += ey(a) * sa_d;
      }
    }
    if (CONS) bC += cw0 * (Ml - divJ) + cwx * (s1x - dPx) + cwy * (s1y - dPy);
  }
  const real inv_m = (real)(1.0 / mi);
#pragma unroll
  for (int a = 0; a < NPOP; ++a) f[a * Np + i] = b[a] * inv_m;
  if (CONS) fC[i] = bC / mi;
}

// ----------------------------------------------------------------------------
// a8: the consistent-mass solve M11 x = b, preconditioned by the lumped mass:
// Richardson sweeps x <- x + w_j (f - A x), A = diag(m)^-1 M11, f = b/m,
// x_0 = f.  With w_j the reciprocal Chebyshev roots on [lambda_min, lambda_max]
// the K-sweep product equals the degree-K Chebyshev iterate.
// (A x)_i = x_i / 2 + sum_j a_ij x_j  (M11_ii / m_i = 1/2 for P1 triangles).
// MODE 0: first sweep (x = f, gathered from f)
// MODE 1: middle sweep (x from xin, write xout)
// MODE 2: last sweep: psi_bar^{n+1} = psi_hat + x_K, then the wall operator
// MODE 3: single sweep (first and last)
// MODE 4: no sweep (K = 0): psi_bar^{n+1} = psi_hat + f, then the wall operator
// In FP32 the same sweeps also advance the composition increment X_C in FP64
// (right-hand side fC, the zeroth h-moment of b/m); its diagonal dlt_j makes
// the column sums sum_i m_i A_ij = m_j exact for the stored a_ij, so every
// sweep keeps sum_i m_i X_C,i = sum_i m_i fC_i to FP64 rounding.  The last
// sweep stores r = (C^n + X_C) - sum_a h_a^{n+1}.
// ----------------------------------------------------------------------------
struct ConsArgs {
  const double* fC;    // [Np]
  const double* xCin;  // [Np]
  double* xCout;       // [Np]
  const double* dlt;   // [Np]
  const double* Cn;    // [Np] composition entering the step
  double* rC;          // [Np] remainder written by the last sweep
  double w;
};

template <typename real, int MODE>
__global__ void __launch_bounds__(BLOCK) k_sweep(int N, int Np, const int* __restrict__ sell_ptr,
                                                const int* __restrict__ sell_col, const real* __restrict__ sell_val,
                                                const real* __restrict__ f, const real* __restrict__ xin,
                                                real* __restrict__ xout, real* __restrict__ pop,
                                                const uint8_t* __restrict__ is_wall, real w, ConsArgs cs) {
  constexpr bool CONS = Conserve<real>::on;
  const int i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= N) return;
  const real* __restrict__ x = (MODE == 0 || MODE == 3) ? f : xin;
  const double* __restrict__ xC = (MODE == 0 || MODE == 3) ? cs.fC : cs.xCin;
  real r[NPOP];
  double rc = 0.0;
  if (MODE != 4) {
#pragma unroll
    for (int a = 0; a < NPOP; ++a) r[a] = (real)0.5 * x[a * Np + i];
    if (CONS) rc = cs.dlt[i] * xC[i];
    const int slice = i >> 6, lane = i & 63;
    const int base = sell_ptr[slice], width = (sell_ptr[slice + 1] - base) >> 6;
    for (int k = 0; k < width; ++k) {
      const int idx = base + (k << 6) + lane;
      const int j = sell_col[idx];
      const real aij = sell_val[idx];
#pragma unroll
      for (int a = 0; a < NPOP; ++a) r[a] += aij * x[a * Np + j];
      if (CONS) rc += (double)aij * xC[j];
    }
#pragma unroll
    for (int a = 0; a < NPOP; ++a) {
      const real xi = x[a * Np + i];
      const real fi = (MODE == 0 || MODE == 3) ? xi : f[a * Np + i];
      r[a] = xi + w * (fi - r[a]);
    }
    if (CONS) {
      const double xi = xC[i];
      const double fi = (MODE == 0 || MODE == 3) ? xi : cs.fC[i];
      rc = xi + cs.w * (fi - rc);
    }
  } else {
#pragma unroll
    for (int a = 0; a < NPOP; ++a) r[a] = f[a * Np + i];
    if (CONS) rc = cs.fC[i];
  }
  if (MODE == 0 || MODE == 1) {
#pragma unroll
    for (int a = 0; a < NPOP; ++a) xout[a * Np + i] = r[a];
    if (CONS) cs.xCout[i] = rc;
    return;
  }
  real s[NPOP];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) s[a] = pop[a * Np + i] + r[a];
  if (is_wall[i]) {
    // wall operator: every opposite pair of g and of h replaced by its mean
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const int b = opp(a);
      if (b > a) {
        const real mg = (real)0.5 * (s[a] + s[b]), mh = (real)0.5 * (s[Q + a] + s[Q + b]);
        s[a] = mg; s[b] = mg; s[Q + a] = mh; s[Q + b] = mh;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < NPOP; ++a) pop[a * Np + i] = s[a];
  if (CONS) {
    double sh = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) sh += (double)s[Q + a];
    cs.rC[i] = (cs.Cn[i] + rc) - sh;
  }
}

// ----------------------------------------------------------------------------
// The sweep on 256-node tiles staged in LDS.  Slots: [0, 256) are the tile's
// own nodes, [256, 256 + halo) its halo (outside neighbours, listed per
// tile).  Matrix rows use 16-bit slots, stored column-major per tile (entry k
// of lane l at tile_off + k*256 + l); padded entries point at the row's own
// slot with weight 0.  Staging by LDS DMA (global_load_lds): the loads write
// LDS directly, so nothing is held in VGPRs while they are in flight and a
// workgroup issues all of its staging (tile, halo, FP64 composition iterate,
// the f values it needs later) before one wait.  Two workgroups per tile, one
// per population set (g: 0..8, h: 9..17), which keeps the LDS of a workgroup
// at 9 populations and lets more tiles be in flight per CU; in FP32 the h
// workgroup also carries the FP64 composition sweep.  Tile values move 16
// bytes per lane; FP32 halo values are 4-byte DMA gathers of 64 entries per
// instruction, FP64 halo values go through registers.  LDS: [9][SLOTS1]
// values, then (FP32) [SLOTS1] doubles.
// ----------------------------------------------------------------------------
template <typename real>
constexpr unsigned sweep_dma_lds_bytes() {
  return Q * SLOTS1 * sizeof(real) + (Conserve<real>::on ? SLOTS1 * 8 : 0);
}

template <typename real, int MODE>
__global__ void __launch_bounds__(BLOCK) k_sweep_dma(int N, int Np, TileArgs ta, const real* __restrict__ tval,
                                                    const real* __restrict__ f, const real* __restrict__ xin,
                                                    real* __restrict__ xout, real* __restrict__ pop,
                                                    const uint8_t* __restrict__ is_wall, real w, ConsArgs cs) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int S = SLOTS1;
  constexpr bool CONS = Conserve<real>::on;
  constexpr bool FIRST = MODE == 0 || MODE == 3;   // iterate = f
  constexpr bool STAGE = MODE != 4;
  // f and the new iterate are streamed with nontemporal accesses (each is
  // touched by one workgroup once per launch)
  constexpr bool NT = true;
  real* xs = reinterpret_cast<real*>(smem);
  double* cxs = reinterpret_cast<double*>(smem + Q * S * sizeof(real));
  const int vb = xcd_block();
  const int t = vb >> 1;
  const bool hset = (vb & 1) != 0;  // block-uniform: this workgroup sweeps h (and, FP32, the composition)
  if (t >= ta.ntiles) return;       // block-uniform
  const int p0 = hset ? Q : 0;
  const int lane = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(lane >> 6);
  const int l = lane & 63;
  const int base = t * TILE;
  const int i = base + lane;
  const bool valid = i < N;
  const int h0 = ta.halo_off[t], nh = ta.halo_off[t + 1] - h0;
  const int e0 = ta.tile_off[t], width = (ta.tile_off[t + 1] - e0) / TILE;
  const real* __restrict__ x = (FIRST ? f : xin) + p0 * Np;
  const double* __restrict__ xC = FIRST ? cs.fC : cs.xCin;
  if (STAGE) {
    // Np is a multiple of 64, so a 16-byte chunk that starts below Np ends inside the array
    constexpr int PER = 16 / sizeof(real);  // values per lane and 16-byte load
#pragma unroll
    for (int c = 0; c < TILE / (64 * PER); ++c)
      if (base + c * 64 * PER + PER * l < Np)
        for (int a = wave; a < Q; a += 4) lds_dma16(x + a * Np + base + c * 64 * PER + PER * l, xs + a * S + c * 64 * PER);
    const int hid0 = l < nh ? ta.halo[h0 + l] : 0;
    const int hid1 = 64 + l < nh ? ta.halo[h0 + 64 + l] : 0;
    for (int a = wave; a < Q; a += 4) {
      if constexpr (sizeof(real) == 4) {
        if (l < nh) lds_dma4(x + a * Np + hid0, xs + a * S + TILE);
        if (64 + l < nh) lds_dma4(x + a * Np + hid1, xs + a * S + TILE + 64);
      } else {
        // 8-byte halo values go through registers (LDS DMA moves at most 4 bytes per gathered lane)
        if (l < nh) xs[a * S + TILE + l] = x[a * Np + hid0];
        if (64 + l < nh) xs[a * S + TILE + 64 + l] = x[a * Np + hid1];
      }
    }
    if (CONS && hset) {
      if (wave < 2) {
        // two doubles per lane; waves 0 and 1 cover tile nodes [0,128) and [128,256)
        if (base + wave * 128 + 2 * l < Np) lds_dma16(xC + base + wave * 128 + 2 * l, cxs + wave * 128);
      } else {
        const int hh = (wave - 2) * 64 + l;
        if (hh < nh) cxs[TILE + hh] = xC[wave == 2 ? hid0 : hid1];
      }
    }
  }
  int sl[MAXW];
  real va[MAXW];
#pragma unroll
  for (int k = 0; k < MAXW; ++k) {
    if (k < width) {
      // ordinary loads: the g and h workgroups of a tile read the same rows
      sl[k] = ta.slot[e0 + k * TILE + lane];
      va[k] = tval[e0 + k * TILE + lane];
    } else {
      sl[k] = lane;
      va[k] = (real)0;
    }
  }
  // the f values of the own node, in flight together with the staging
  real fr[Q];
  double fCi = 0.0, dlti = 0.0;
  if (!FIRST && valid) {
#pragma unroll
    for (int a = 0; a < Q; ++a) fr[a] = ld_stream<NT>(&f[(p0 + a) * Np + i]);
    if (CONS && hset) fCi = cs.fC[i];
  }
  if (CONS && STAGE && hset && valid) dlti = cs.dlt[i];
  if (STAGE) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's LDS DMA has landed
    __syncthreads();
  }
  if (!valid) return;
  real r[Q];
  double rc = 0.0;
  if (STAGE) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const real xi = xs[a * S + lane];
      real acc = (real)0.5 * xi;
#pragma unroll
      for (int k = 0; k < MAXW; ++k)
        if (k < width) acc += va[k] * xs[a * S + sl[k]];
      r[a] = xi + w * ((FIRST ? xi : fr[a]) - acc);
      if (MODE == 0 || MODE == 1) st_stream<NT>(r[a], &xout[(p0 + a) * Np + i]);
    }
    if (CONS && hset) {
      const double xco = cxs[lane];
      double acc = dlti * xco;
#pragma unroll
      for (int k = 0; k < MAXW; ++k)
        if (k < width) acc += (double)va[k] * cxs[sl[k]];
      rc = xco + cs.w * ((FIRST ? xco : fCi) - acc);
    }
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) r[a] = fr[a];
    rc = fCi;
  }
  if (MODE == 0 || MODE == 1) {
    if (CONS && hset) st_stream<NT>(rc, &cs.xCout[i]);
    return;
  }
  real s[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) s[a] = pop[(p0 + a) * Np + i] + r[a];
  if (is_wall[i]) {
    // wall operator: every opposite pair of this population set replaced by its mean
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const int b = opp(a);
      if (b > a) {
        const real m = (real)0.5 * (s[a] + s[b]);
        s[a] = m; s[b] = m;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < Q; ++a) pop[(p0 + a) * Np + i] = s[a];
  if (CONS && hset) {
    double sh = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) sh += (double)s[a];
    cs.rC[i] = (cs.Cn[i] + rc) - sh;
  }
}

// ----------------------------------------------------------------------------
// init: psi_bar^0 = psi_eq(C, u, p), then the wall operator
// ----------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_init(int N, int Np, StepParams P, const double* __restrict__ C,
                                               const double* __restrict__ U, const double* __restrict__ Pr,
                                               const uint8_t* __restrict__ is_wall, real* __restrict__ pop,
                                               double* __restrict__ rC) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= N) return;
  const double c = C[i], ux = U[2 * i], uy = U[2 * i + 1], p = Pr[i];
  const double rho = c * P.rho_l + (1.0 - c) * P.rho_v, uu = ux * ux + uy * uy;
  double s[NPOP];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy;
    const double poly = eu + 1.5 * eu * eu - 0.5 * uu;
    s[a] = wq(a) * (p + rho * poly);
    s[Q + a] = wq(a) * c * (1.0 + 3.0 * poly);
  }
  if (is_wall[i]) {
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const int b = opp(a);
      if (b > a) {
        const double mg = 0.5 * (s[a] + s[b]), mh = 0.5 * (s[Q + a] + s[Q + b]);
        s[a] = mg; s[b] = mg; s[Q + a] = mh; s[Q + b] = mh;
      }
    }
  }
  double sh = 0.0;
#pragma unroll
  for (int a = 0; a < NPOP; ++a) {
    const real v = (real)s[a];
    pop[a * Np + i] = v;
    if (a >= Q) sh += (double)v;
  }
  if (Conserve<real>::on) rC[i] = c - sh;
}

// Wetting potential handed over in device memory (caller node order): flags[0]
// is set if any value is non-finite, flags[1] if a wall node has a nonzero one.
// Every thread that sets a flag stores the same value.
__global__ void __launch_bounds__(BLOCK) k_wetting_check(int N, const int* __restrict__ node_perm,
                                                        const uint8_t* __restrict__ is_wall,
                                                        const double* __restrict__ omega, int32_t* __restrict__ flags) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= N) return;
  const double v = omega[node_perm[k]];
  if (!isfinite(v)) flags[0] = 1;
  if (is_wall[k] && v != 0.0) flags[1] = 1;
}

// phi_c / kappa = Omega_c sqrt(2 kappa beta) / kappa at wall nodes (eq. bc2),
// 0 elsewhere, in internal order; the same operations as the host path
__global__ void __launch_bounds__(BLOCK) k_wetting_bc(int N, const int* __restrict__ node_perm,
                                                     const uint8_t* __restrict__ is_wall,
                                                     const double* __restrict__ omega, double sq, double kappa,
                                                     double* __restrict__ bc) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= N) return;
  const double v = omega[node_perm[k]];
  bc[k] = (is_wall[k] && v != 0.0) ? __ddiv_rn(__dmul_rn(v, sq), kappa) : 0.0;
}

// a nodal field from internal to caller order; rho = C rho_l + (1 - C) rho_v
// when to_rho is set (unfused, as on the host)
__global__ void __launch_bounds__(BLOCK) k_field_to_caller(int N, const int* __restrict__ node_perm,
                                                          const double* __restrict__ src, double* __restrict__ dst,
                                                          int to_rho, double rho_l, double rho_v) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= N) return;
  const double v = src[k];
  dst[node_perm[k]] = to_rho ? __dadd_rn(__dmul_rn(v, rho_l), __dmul_rn(__dsub_rn(1.0, v), rho_v)) : v;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename real>
__global__ void __launch_bounds__(BLOCK) k_to_double(int n, const real* __restrict__ in, double* __restrict__ out) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

}  // namespace felbm
