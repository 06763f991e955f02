// HIP kernels (gfx950) of one FE-LBM time step in 3-D: D3Q19 populations g, h
// on linear tetrahedra, the paper's own setting (arXiv:1708.04678, Sec. II.A:
// D3Q19; Sec. II.C: tetrahedral elements).  The same steps as the 2-D
// kernels with the tetrahedral forms; all gathers are global (node-centric,
// one thread per output, no atomics), the element data in structure-of-arrays
// order.
//
// Data layout (device):
//   populations  per set [5][Np][4] (populations 4q..4q+3 of node j at [q][j],
//                slot 19 unused), the g set then the h set, Np = N rounded to 64
//   elements     tet int32 [4][E]; shape-function gradients grad N_1 .. grad N_3
//                ([9][E], grad N_0 = -(grad N_1 + grad N_2 + grad N_3) formed
//                in the kernel): FP64 steps as such, FP32 steps from the FP64
//                geometry record [10][E] = (V, grad N_1 .. grad N_3)
//   field operators: the patch Laplacian of C over the 2-ring (sliced ELL,
//                weights / patch volume) with the wall faces of each patch
//                (CSR); the element Laplacian of mu ([4][E] vertices across
//                the faces, [7][E] weights)
//   mass matrix  diag(m)^-1 M11 off-diagonal part, sliced ELL (slice 64);
//                its diagonal is M11_ii / m_i = 2/5 for P1 tetrahedra
//   right-hand side: incident-element weights [4][slots] and patch moments
//                [9][slots] in sliced ELL; element force parameters [13][E]
//   solve vectors (the right-hand side f and the sweep iterates): the same
//                layout as the populations
#pragma once

#include "common.hpp"

namespace felbm3d {

using felbm::BLOCK;
using felbm::CS2;
using felbm::StepParams;
using felbm::xcd_block;

constexpr int Q = 19;
constexpr int NPOP = 38;

// D3Q19: rest, the six axis directions (+x, -x, +y, -y, +z, -z), then the
// twelve face diagonals of the (x,y), (x,z), (y,z) planes in the order
// (+,+), (-,-), (+,-), (-,+)
__host__ __device__ constexpr int ex(int a) {
  return a == 1 ? 1 : a == 2 ? -1 : (a >= 7 && a <= 14) ? ((a == 7 || a == 9 || a == 11 || a == 13) ? 1 : -1) : 0;
}
__host__ __device__ constexpr int ey(int a) {
  return a == 3 ? 1 : a == 4 ? -1
       : (a >= 7 && a <= 10) ? ((a == 7 || a == 10) ? 1 : -1)
       : (a >= 15) ? ((a == 15 || a == 17) ? 1 : -1) : 0;
}
__host__ __device__ constexpr int ez(int a) {
  return a == 5 ? 1 : a == 6 ? -1
       : (a >= 11 && a <= 14) ? ((a == 11 || a == 14) ? 1 : -1)
       : (a >= 15) ? ((a == 15 || a == 18) ? 1 : -1) : 0;
}
__host__ __device__ constexpr double wq(int a) { return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr int opp(int a) {
  return a == 0 ? 0 : (a < 7 ? ((a & 1) ? a + 1 : a - 1) : (((a - 7) & 1) ? a - 1 : a + 1));
}

// The populations and the solve vectors hold each population set as five
// groups of four populations per node, so that the 19 values of a gathered
// neighbour arrive in five 16-byte (FP64: 32-byte) loads instead of nineteen
// 4-byte ones.
constexpr int QS = 20;  // slots per node and set
template <typename real>
struct Quad4;
template <>
struct Quad4<float> {
  using type = float4;
};
template <>
struct Quad4<double> {
  using type = double4;
};
// v[0..19] <- the set at node j (v[19] is the unused slot)
template <typename real>
__device__ __forceinline__ void load_set(const real* __restrict__ base, int j, int Np, real* v) {
  using V4 = typename Quad4<real>::type;
  const V4* b4 = reinterpret_cast<const V4*>(base);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const V4 t = b4[(size_t)q * Np + j];
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
}
// the set at node i <- v[0..18]; the unused slot is written as 0
template <typename real>
__device__ __forceinline__ void store_set(real* __restrict__ base, int i, int Np, const real* v) {
  using V4 = typename Quad4<real>::type;
  V4* b4 = reinterpret_cast<V4*>(base);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    V4 t;
    t.x = v[4 * q];
    t.y = v[4 * q + 1];
    t.z = v[4 * q + 2];
    t.w = q < 4 ? v[4 * q + 3] : (real)0;
    b4[(size_t)q * Np + i] = t;
  }
}

// the same for vectors touched once per launch (the right-hand side read by a
// sweep at its own node, the new iterate): nontemporal accesses.  Used by the
// FP32 sweeps only: they ran 2 % faster with them, the FP64 sweeps 1 % slower.
template <typename real>
struct NatV4;
template <>
struct NatV4<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct NatV4<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};
template <typename real>
__device__ __forceinline__ void load_set_nt(const real* __restrict__ base, int j, int Np, real* v) {
  using V = typename NatV4<real>::type;
  const V* b4 = reinterpret_cast<const V*>(base);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const V t = __builtin_nontemporal_load(b4 + (size_t)q * Np + j);
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
}
template <typename real>
__device__ __forceinline__ void store_set_nt(real* __restrict__ base, int i, int Np, const real* v) {
  using V = typename NatV4<real>::type;
  V* b4 = reinterpret_cast<V*>(base);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    V t;
    t.x = v[4 * q];
    t.y = v[4 * q + 1];
    t.z = v[4 * q + 2];
    t.w = q < 4 ? v[4 * q + 3] : (real)0;
    __builtin_nontemporal_store(t, b4 + (size_t)q * Np + i);
  }
}

constexpr int NRED3 = 6;  // same record as the 2-D reductions (band entries stay 0)

// FP32 precision form: the composition is carried in FP64 beside the float
// populations, C = sum_a h_a + r with a per-node FP64 remainder r.  Its
// increment is the zeroth moment of the h right-hand side formed in FP64 from
// the moment identities of the equilibrium (sum_a Phi_h = M lap mu,
// sum_a e_a Phi_h = c_s^2 X + M lap mu u_bar) and from the first and second
// moments J, Pi of the collided h; it is solved by the same Chebyshev steps in
// FP64 with a diagonal that gives the stored float matrix exact mass-weighted
// column sums, and the last sweep stores r = (C^n + X_C) - sum_a h_a^{n+1}.
// Each element's moment terms are formed once (by one thread), so all of its
// vertices see the same values and the mass balance holds to FP64 rounding.
// Every pointer is null in FP64 (and em in the field read-back).
struct Cons3 {
  double* r;           // [N] remainder
  double* jp;          // [9][Np] J (x, y, z), Pi (xx, yy, zz, xy, xz, yz) of the collided h
  double* em;          // [4][E] the element's FP64 contribution to the zeroth moment at each
                       // of its vertices l: V (dt/4 s0 + dt^2/2 grad N_l . s1), with
                       // s0 = d - sum_v grad N_v . J_v, s1 = c_s^2 X + d u_bar - sum_v Pi_v grad N_v
  const double* geo;   // [10][E] V and grad N_1 .. grad N_3 in FP64
  double* fC;          // [Np] right-hand side / m
  const double* xCin;  // [Np] iterate in
  double* xCout;       // [Np] iterate out
  const double* dlt;   // [N] diagonal of the FP64 sweeps
  const double* Cn;    // [N] composition at the start of the step
  double w;            // Chebyshev step of the current sweep
};

// a1 + a6: moments, relaxation time, equilibria and BGK collision; block partials of the reductions
template <typename real, bool COLLIDE>
__global__ void __launch_bounds__(BLOCK) k3_moments(real* __restrict__ pop, int N, int Np, StepParams P,
                                                   double* __restrict__ Cn, real* __restrict__ pn,
                                                   real* __restrict__ un, const double* __restrict__ mass,
                                                   double* __restrict__ partials, Cons3 cs) {
  constexpr bool CONS = sizeof(real) == 4;
  const int blk = xcd_block();
  const int i = blk * BLOCK + threadIdx.x;
  double red[NRED3] = {0, 0, 0, 0, 0, 0};
  if (i < N) {
    double C = CONS ? cs.r[i] : 0.0;
    real p = 0, jx = 0, jy = 0, jz = 0;
    {
      real gv[QS], hv[QS];
      load_set(pop, i, Np, gv);
      load_set(pop + (size_t)QS * Np, i, Np, hv);
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const real g = gv[a];
        C += (double)hv[a];
        p += g;
      if (ex(a)) jx += ex(a) > 0 ? g : -g;
      if (ey(a)) jy += ey(a) > 0 ? g : -g;
        if (ez(a)) jz += ez(a) > 0 ? g : -g;
      }
    }
    const real rho = (real)(C * P.rho_l + (1.0 - C) * P.rho_v);
    const real ux = (real)3 * jx / rho, uy = (real)3 * jy / rho, uz = (real)3 * jz / rho;
    Cn[i] = C;
    pn[i] = p;
    un[i] = ux;
    un[Np + i] = uy;
    un[2 * Np + i] = uz;
    const real uu = ux * ux + uy * uy + uz * uz;
    if (COLLIDE) {
      const real tau = (real)(1.0 / (C * P.inv_tau_l + (1.0 - C) * P.inv_tau_v));
      const real om = (real)1 / (tau + (real)0.5);
      const real Cr = (real)C;
      double J[3] = {0, 0, 0}, Pi[6] = {0, 0, 0, 0, 0, 0};
      using V4 = typename Quad4<real>::type;
      V4* pg = reinterpret_cast<V4*>(pop);
      V4* ph = reinterpret_cast<V4*>(pop + (size_t)QS * Np);
      // one group of four populations at a time (read again: the first read is in cache)
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const V4 g4 = pg[(size_t)q * Np + i], h4 = ph[(size_t)q * Np + i];
        const real gq[4] = {g4.x, g4.y, g4.z, g4.w}, hq[4] = {h4.x, h4.y, h4.z, h4.w};
        real go[4] = {0, 0, 0, 0}, ho[4] = {0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int a = 4 * q + c;
          if (a >= Q) continue;
          const real eu = (real)ex(a) * ux + (real)ey(a) * uy + (real)ez(a) * uz;
          const real poly = eu + (real)1.5 * eu * eu - (real)0.5 * uu;
          const real geq = (real)wq(a) * (p + rho * poly);
          const real heq = (real)wq(a) * Cr * ((real)1 + (real)3 * poly);
          const real g = gq[c], h = hq[c];
          const real hn = h - om * (h - heq);
          go[c] = g - om * (g - geq);
          ho[c] = hn;
          if (CONS) {
            const double hd = (double)hn;
            if (ex(a)) J[0] += ex(a) * hd;
            if (ey(a)) J[1] += ey(a) * hd;
            if (ez(a)) J[2] += ez(a) * hd;
            if (ex(a)) Pi[0] += hd;
            if (ey(a)) Pi[1] += hd;
            if (ez(a)) Pi[2] += hd;
            if (ex(a) && ey(a)) Pi[3] += ex(a) * ey(a) * hd;
            if (ex(a) && ez(a)) Pi[4] += ex(a) * ez(a) * hd;
            if (ey(a) && ez(a)) Pi[5] += ey(a) * ez(a) * hd;
          }
        }
        pg[(size_t)q * Np + i] = V4{go[0], go[1], go[2], go[3]};
        ph[(size_t)q * Np + i] = V4{ho[0], ho[1], ho[2], ho[3]};
      }
      if (CONS) {
#pragma unroll
        for (int c = 0; c < 3; ++c) cs.jp[c * Np + i] = J[c];
#pragma unroll
        for (int c = 0; c < 6; ++c) cs.jp[(3 + c) * Np + i] = Pi[c];
      }
    }
    const double uud = (double)uu;
    red[0] = mass[i] * C;
    red[1] = (C * P.rho_l + (1.0 - C) * P.rho_v) * uud;
    red[2] = sqrt(uud);
    red[5] = (isfinite(C) && isfinite((double)p) && isfinite(uud)) ? 0.0 : 1.0;
    if (red[5] != 0.0) red[2] = 0.0;
  }
  felbm::block_reduce_store<NRED3>(red, 2, partials, gridDim.x, blk);
}

// Outward flux through a wall face from eq. bc2 (n into the fluid):
// -int (phi_c/kappa)(C - C^2) dA with r = phi_c/kappa and C linear on the
// triangle, exact: int lambda_i lambda_j = A (1 + delta_ij)/12 and
// int lambda_i lambda_j lambda_k = A/10, A/30, A/60 for three, two, no equal
// indices.
__device__ __forceinline__ double wall_flux3(const double (&C)[3], const double (&r)[3], double area) {
  double lin = 0.0, cub = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      lin += r[i] * C[j] * (i == j ? 2.0 : 1.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double wgt = (i == j && j == k) ? 6.0 : ((i == j || j == k || i == k) ? 2.0 : 1.0);
        cub += r[i] * C[j] * C[k] * wgt;
      }
    }
  return -area * (lin * (1.0 / 12.0) - cub * (1.0 / 60.0));
}

// a3 as a precomputed operator.  The patch Laplacian of C (eqn:lapl_int_mp:
// averaged element gradients across the interior outer faces of the patch,
// the wetting flux of eq. bc2 over its wall faces) is linear in the nodal C of
// the patch and of the vertices across its outer faces, apart from the wall
// terms; with the weights divided by the patch volume V_k on the host,
//   lap C_k = sum_j w_kj (C_j - C_k) + sum_{wall faces f of the patch} F_BC(f) / V_k
// (difference form: sum_j w_kj = 0, so a constant field gives exactly 0).
// Rows in sliced ELL (slice 64, entry q of lane l at base + 64 q + l, padding
// pointing at the node itself with weight 0); the wall faces of each patch (those
// opposite the node and those containing it) in a CSR list of node triples
// [3][L] and area / V_k.  Values and arithmetic in FP64, weights in wreal.
template <typename wreal>
__global__ void __launch_bounds__(BLOCK) k3_lapC_mu_op(int N, const int* __restrict__ lop_ptr,
                                                      const int* __restrict__ lop_col, const wreal* __restrict__ lop_w,
                                                      const int* __restrict__ wl_ptr, const int* __restrict__ wl_face,
                                                      const double* __restrict__ wl_scale, int L,
                                                      const double* __restrict__ Cn, const double* __restrict__ bc,
                                                      StepParams P, double* __restrict__ lapC, double* __restrict__ mu) {
  const int i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= N) return;
  const int slice = i >> 6, lane = i & 63;
  const int base = lop_ptr[slice], width = (lop_ptr[slice + 1] - base) >> 6;
  const double Ci = Cn[i];
  double acc = 0.0;
  for (int q = 0; q < width; ++q) {
    const int idx = base + (q << 6) + lane;
    acc += (double)lop_w[idx] * (Cn[lop_col[idx]] - Ci);
  }
  for (int q = wl_ptr[i]; q < wl_ptr[i + 1]; ++q) {
    double Cf[3], rf[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int n = wl_face[c * L + q];
      Cf[c] = Cn[n];
      rf[c] = bc[n];
    }
    acc += wall_flux3(Cf, rf, wl_scale[q]);
  }
  lapC[i] = acc;
  mu[i] = 2.0 * P.beta * Ci * (Ci - 1.0) * (2.0 * Ci - 1.0) - P.kappa * acc;
}

// a4 + a2 + a5: the element Laplacian of mu (Sec. II.D: -3/2 sum_l grad N_l .
// (grad mu_T + grad mu_T'(l)) over the interior faces, zero on wall faces) as
// a precomputed operator on mu at the element's vertices and at the four
// vertices across its faces,
//   lap mu_T = sum_{v=1..3} a_v (mu_v - mu_0) + sum_l b_l (mu_opp(l) - mu_0)
// (a wall face contributes nothing: its opposite slot points at vertex 0 with
// weight 0); then the element gradients of C and p and the element's force
// parameters at the barycentric values (eq:G, eq:H): for the g set
// A = (rho_l - rho_v) c_s^2 grad C_T and B = mu_bar grad C_T, for the h set
// X = grad C_T - C_bar / (rho_bar c_s^2) (grad p_T - mu_bar grad C_T) and
// d = M lap mu_T; both with u_bar.  Stored [13][E] as (u_bar, A, B, X, d).
// The shape-function gradients grad N_1 .. grad N_3 are read in FP64 (FP32
// steps: from the geometry record) and grad N_0 = -(grad N_1 + grad N_2 +
// grad N_3) formed in the order of the mesh preparation; every force
// parameter is rounded to the working precision.
template <typename real, typename wreal>
__global__ void __launch_bounds__(BLOCK) k3_lapmu_force_op(int E, int Np, const int* __restrict__ tet,
                                                          const int* __restrict__ eopp, const wreal* __restrict__ ew,
                                                          const double* __restrict__ grad,
                                                          const double* __restrict__ Cn, const double* __restrict__ mu,
                                                          const real* __restrict__ pn, const real* __restrict__ un,
                                                          StepParams P, double* __restrict__ lapmu,
                                                          real* __restrict__ fpar, Cons3 cs) {
  constexpr bool CONS = sizeof(real) == 4;
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= E) return;
  int v[4];
  double Cv[4], mv[4];
  real pv[4];
  double Cb = 0.0, mub = 0.0;
  real ubx = 0, uby = 0, ubz = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    v[t] = tet[t * E + e];
    Cv[t] = Cn[v[t]];
    mv[t] = mu[v[t]];
    pv[t] = pn[v[t]];
    Cb += Cv[t];
    mub += mv[t];
    ubx += un[v[t]];
    uby += un[Np + v[t]];
    ubz += un[2 * Np + v[t]];
  }
  double lm = (double)ew[e] * (mv[1] - mv[0]) + (double)ew[E + e] * (mv[2] - mv[0]) +
              (double)ew[2 * E + e] * (mv[3] - mv[0]);
#pragma unroll
  for (int l = 0; l < 4; ++l) lm += (double)ew[(3 + l) * E + e] * (mu[eopp[l * E + e]] - mv[0]);
  lapmu[e] = lm;
  // FP64 shape-function gradients (rows of vertex 1..3), grad N_0 from their sum
  const double* __restrict__ g = CONS ? cs.geo + E : grad;
  double gxd[4], gyd[4], gzd[4];
#pragma unroll
  for (int t = 1; t < 4; ++t) {
    gxd[t] = g[(3 * t - 3) * E + e];
    gyd[t] = g[(3 * t - 2) * E + e];
    gzd[t] = g[(3 * t - 1) * E + e];
  }
  gxd[0] = -(gxd[1] + gxd[2] + gxd[3]);
  gyd[0] = -(gyd[1] + gyd[2] + gyd[3]);
  gzd[0] = -(gzd[1] + gzd[2] + gzd[3]);
  double gCx = 0.0, gCy = 0.0, gCz = 0.0;
  real gpx = 0, gpy = 0, gpz = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const real gx = (real)gxd[t], gy = (real)gyd[t], gz = (real)gzd[t];
    gCx += Cv[t] * (double)gx;
    gCy += Cv[t] * (double)gy;
    gCz += Cv[t] * (double)gz;
    gpx += pv[t] * gx;
    gpy += pv[t] * gy;
    gpz += pv[t] * gz;
  }
  Cb *= 0.25;
  mub *= 0.25;
  const real drho_cs2 = (real)(CS2 * (P.rho_l - P.rho_v));
  const real rhob = (real)(Cb * P.rho_l + (1.0 - Cb) * P.rho_v);
  const real bx = (real)(mub * gCx), by = (real)(mub * gCy), bz = (real)(mub * gCz);
  const real coef = (real)Cb / (rhob * (real)CS2);
  real* __restrict__ o = fpar + e;
  o[0] = ubx * (real)0.25;
  o[E] = uby * (real)0.25;
  o[2 * E] = ubz * (real)0.25;
  o[3 * E] = drho_cs2 * (real)gCx;
  o[4 * E] = drho_cs2 * (real)gCy;
  o[5 * E] = drho_cs2 * (real)gCz;
  o[6 * E] = bx;
  o[7 * E] = by;
  o[8 * E] = bz;
  o[9 * E] = (real)gCx - coef * (gpx - bx);
  o[10 * E] = (real)gCy - coef * (gpy - by);
  o[11 * E] = (real)gCz - coef * (gpz - bz);
  o[12 * E] = (real)(P.mobility * lm);
  if (CONS && cs.em) {
    // FP64 moment terms of this element (FP64 geometry, vertex order 0..3)
    const double *gx = gxd, *gy = gyd, *gz = gzd;
    double GCx = 0.0, GCy = 0.0, GCz = 0.0, Gpx = 0.0, Gpy = 0.0, Gpz = 0.0, uxd = 0.0, uyd = 0.0, uzd = 0.0;
    double divJ = 0.0, Dx = 0.0, Dy = 0.0, Dz = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      GCx += Cv[t] * gx[t];
      GCy += Cv[t] * gy[t];
      GCz += Cv[t] * gz[t];
      Gpx += (double)pv[t] * gx[t];
      Gpy += (double)pv[t] * gy[t];
      Gpz += (double)pv[t] * gz[t];
      uxd += (double)un[v[t]];
      uyd += (double)un[Np + v[t]];
      uzd += (double)un[2 * Np + v[t]];
      const double* q = cs.jp + v[t];
      const double Jx = q[0], Jy = q[(size_t)Np], Jz = q[2 * (size_t)Np];
      const double Pxx = q[3 * (size_t)Np], Pyy = q[4 * (size_t)Np], Pzz = q[5 * (size_t)Np];
      const double Pxy = q[6 * (size_t)Np], Pxz = q[7 * (size_t)Np], Pyz = q[8 * (size_t)Np];
      divJ += gx[t] * Jx + gy[t] * Jy + gz[t] * Jz;
      Dx += Pxx * gx[t] + Pxy * gy[t] + Pxz * gz[t];
      Dy += Pxy * gx[t] + Pyy * gy[t] + Pyz * gz[t];
      Dz += Pxz * gx[t] + Pyz * gy[t] + Pzz * gz[t];
    }
    uxd *= 0.25;
    uyd *= 0.25;
    uzd *= 0.25;
    const double rhod = Cb * P.rho_l + (1.0 - Cb) * P.rho_v;
    const double cf = Cb / (rhod * CS2);
    const double Ml = P.mobility * lm;
    const double s0 = Ml - divJ;
    const double s1x = CS2 * (GCx - cf * (Gpx - mub * GCx)) + Ml * uxd - Dx;
    const double s1y = CS2 * (GCy - cf * (Gpy - mub * GCy)) + Ml * uyd - Dy;
    const double s1z = CS2 * (GCz - cf * (Gpz - mub * GCz)) + Ml * uzd - Dz;
    const double V = cs.geo[e], c1 = 0.25 * P.dt, c2 = 0.5 * P.dt * P.dt;
#pragma unroll
    for (int l = 0; l < 4; ++l) cs.em[l * E + e] = V * (c1 * s0 + c2 * (gx[l] * s1x + gy[l] * s1y + gz[l] * s1z));
  }
}

// a5 + a7: the Galerkin right-hand side (eq:galerkin_lbm) divided by m_i,
// one thread per (node, population set).  With weights alpha = (dt/4) V_T / m_i
// and beta = (dt^2/2) V_T grad N_i|_T / m_i of each incident element and the
// patch moments G_ij = (dt/4) sum_T V_T grad N_j / m_i and
// S_ij = (dt^2/2) sum_T V_T (grad N_i grad N_j^T) / m_i (held as xx, yy, zz and
// the doubled symmetric xy, xz, yz), both precomputed from the geometry:
//   f_{a,i} = sum_T (alpha + e_a . beta) Phi_{a,T}
//           - sum_j psi_hat_{a,j} (e_a . G_ij + e_a . S_ij e_a),
// which is b_{a,i}/m_i with q_{a,T} = Phi_{a,T} - e_a . sum_v psi_hat_{a,v} grad N_v
// regrouped by node (each psi_hat value is gathered once per patch node instead
// of once per incident element).  The first half of the grid computes the g
// set, the second half the h set, four 64-node slices per block.  Element weights and patch moments are in
// sliced-ELL order (slice of 64 nodes, entry k of lane l at base + 64 k + l).
template <typename real>
__global__ void __launch_bounds__(BLOCK) k3_rhs(int N, int Np, int E, const int* __restrict__ inc_ptr,
                                               const int* __restrict__ inc_e, const real* __restrict__ inc_w,
                                               int inc_slots, const real* __restrict__ fpar,
                                               const int* __restrict__ pair_ptr, const int* __restrict__ pair_col,
                                               const real* __restrict__ pair_v, int pair_slots,
                                               const real* __restrict__ pop, real* __restrict__ f,
                                               const double* __restrict__ mass, Cons3 cs) {
  constexpr bool CONS = sizeof(real) == 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int blk = xcd_block(), half = gridDim.x >> 1;
  const bool hset = blk >= half;
  const int slice = (blk - (hset ? half : 0)) * 4 + wave;
  const int i = (slice << 6) + lane;
  if (i >= N) return;
  real b[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) b[a] = (real)0;
  double bC = 0.0;
  {
    const int base = inc_ptr[slice], width = (inc_ptr[slice + 1] - base) >> 6;
    for (int k = 0; k < width; ++k) {
      const int idx = base + (k << 6) + lane;
      const int el = inc_e[idx];
      if (el < 0) continue;
      const int e = el >> 2;
      const real al = inc_w[idx], btx = inc_w[inc_slots + idx], bty = inc_w[2 * inc_slots + idx],
                 btz = inc_w[3 * inc_slots + idx];
      const real ux = fpar[e], uy = fpar[E + e], uz = fpar[2 * E + e];
      const real uu = ux * ux + uy * uy + uz * uz;
      if (!hset) {
        const real Ax = fpar[3 * E + e], Ay = fpar[4 * E + e], Az = fpar[5 * E + e];
        const real Bx = fpar[6 * E + e], By = fpar[7 * E + e], Bz = fpar[8 * E + e];
        const real uA = ux * Ax + uy * Ay + uz * Az, uB = ux * Bx + uy * By + uz * Bz;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const real exa = (real)ex(a), eya = (real)ey(a), eza = (real)ez(a);
          const real eu = exa * ux + eya * uy + eza * uz;
          const real G = (real)wq(a) * ((real)1 + (real)3 * eu + (real)4.5 * eu * eu - (real)1.5 * uu);
          const real Phi = (exa * Ax + eya * Ay + eza * Az - uA) * (G - (real)wq(a)) +
                           (exa * Bx + eya * By + eza * Bz - uB) * G;
          b[a] += (al + exa * btx + eya * bty + eza * btz) * Phi;
        }
      } else {
        if (CONS) bC += cs.em[(el & 3) * E + e];  // FP64 zeroth moment, divided by m_i below
        const real Xx = fpar[9 * E + e], Xy = fpar[10 * E + e], Xz = fpar[11 * E + e], d = fpar[12 * E + e];
        const real uX = ux * Xx + uy * Xy + uz * Xz;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const real exa = (real)ex(a), eya = (real)ey(a), eza = (real)ez(a);
          const real eu = exa * ux + eya * uy + eza * uz;
          const real G = (real)wq(a) * ((real)1 + (real)3 * eu + (real)4.5 * eu * eu - (real)1.5 * uu);
          b[a] += (al + exa * btx + eya * bty + eza * btz) * ((exa * Xx + eya * Xy + eza * Xz - uX + d) * G);
        }
      }
    }
  }
  const real* __restrict__ ps = pop + (hset ? (size_t)QS * Np : 0);
  {
    const int base = pair_ptr[slice], width = (pair_ptr[slice + 1] - base) >> 6;
    for (int k = 0; k < width; ++k) {
      const int idx = base + (k << 6) + lane;
      const int j = pair_col[idx];
      const real Gx = pair_v[idx], Gy = pair_v[pair_slots + idx], Gz = pair_v[2 * pair_slots + idx];
      const real Sxx = pair_v[3 * pair_slots + idx], Syy = pair_v[4 * pair_slots + idx],
                 Szz = pair_v[5 * pair_slots + idx], Sxy = pair_v[6 * pair_slots + idx],
                 Sxz = pair_v[7 * pair_slots + idx], Syz = pair_v[8 * pair_slots + idx];
      real v[QS];
      load_set(ps, j, Np, v);
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const real exa = (real)ex(a), eya = (real)ey(a), eza = (real)ez(a);
        const real c = exa * Gx + eya * Gy + eza * Gz + exa * exa * Sxx + eya * eya * Syy + eza * eza * Szz +
                       exa * eya * Sxy + exa * eza * Sxz + eya * eza * Syz;
        b[a] -= c * v[a];
      }
    }
  }
  store_set(f + (hset ? (size_t)QS * Np : 0), i, Np, b);
  if (CONS && hset) cs.fC[i] = bC / mass[i];
}

// a8: Richardson sweeps with the reciprocal Chebyshev roots on [1/5, 1] (the
// spectrum of diag(m)^-1 M11 for P1 tetrahedra), x0 = f; (A x)_i = 2/5 x_i +
// sum_j a_ij x_j.  MODE 0 first (x = f), 1 middle, 2 last (+ psi_hat and the
// wall operator), 3 single, 4 none (psi_hat + f).  One thread per (node,
// population set): the first half of the grid sweeps the 19 g populations, the
// second half the 19 h populations (opposite pairs stay within one thread for
// the wall operator), each block four 64-node matrix slices.  Keeping a block
// on one set measured 2.3x faster than splitting a block's waves between the
// sets.
template <typename real, int MODE>
__global__ void __launch_bounds__(BLOCK) k3_sweep(int N, int Np, const int* __restrict__ sell_ptr,
                                                 const int* __restrict__ sell_col, const real* __restrict__ sell_val,
                                                 const real* __restrict__ f, const real* __restrict__ xin,
                                                 real* __restrict__ xout, real* __restrict__ pop,
                                                 const uint8_t* __restrict__ is_wall, real w, Cons3 cs) {
  constexpr bool CONS = sizeof(real) == 4;
  constexpr bool FIRST = MODE == 0 || MODE == 3;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = xcd_block(), half = gridDim.x >> 1;
  const bool hset = b >= half;
  const int slice = (b - (hset ? half : 0)) * 4 + wave;
  const int i = (slice << 6) + lane;
  if (i >= N) return;
  const size_t off = hset ? (size_t)QS * Np : 0;  // the set in the populations and solve vectors
  const real* __restrict__ fs = f + off;
  const real* __restrict__ x = (MODE == 0 || MODE == 3) ? fs : xin + off;
  real r[QS], v[QS];
  // the FP64 composition sweep rides with the h set
  const bool comp = CONS && hset;
  const double* __restrict__ xC = FIRST ? cs.fC : cs.xCin;
  double rc = 0.0;
  if (MODE != 4) {
    load_set(x, i, Np, v);
#pragma unroll
    for (int a = 0; a < Q; ++a) r[a] = (real)0.4 * v[a];
    double accC = comp ? cs.dlt[i] * xC[i] : 0.0;
    const int base = sell_ptr[slice], width = (sell_ptr[slice + 1] - base) >> 6;
    for (int k = 0; k < width; ++k) {
      const int idx = base + (k << 6) + lane;
      const int j = sell_col[idx];
      const real aij = sell_val[idx];
      load_set(x, j, Np, v);
#pragma unroll
      for (int a = 0; a < Q; ++a) r[a] += aij * v[a];
      if (comp) accC += (double)aij * xC[j];
    }
    // x_i and f_i again (the first read is in cache), so that they hold no
    // registers through the gather
    load_set(x, i, Np, v);
    if (FIRST) {
#pragma unroll
      for (int a = 0; a < Q; ++a) r[a] = v[a] + w * (v[a] - r[a]);
    } else {
      real fv[QS];
      if constexpr (CONS) load_set_nt(fs, i, Np, fv);
      else load_set(fs, i, Np, fv);
#pragma unroll
      for (int a = 0; a < Q; ++a) r[a] = v[a] + w * (fv[a] - r[a]);
    }
    if (comp) {
      const double xci = xC[i];
      rc = xci + cs.w * ((FIRST ? xci : cs.fC[i]) - accC);
    }
  } else {
    load_set(fs, i, Np, r);
    if (comp) rc = cs.fC[i];
  }
  if (MODE == 0 || MODE == 1) {
    if constexpr (CONS) store_set_nt(xout + off, i, Np, r);
    else store_set(xout + off, i, Np, r);
    if (comp) cs.xCout[i] = rc;
    return;
  }
  real* __restrict__ ps = pop + off;
  load_set(ps, i, Np, v);
#pragma unroll
  for (int a = 0; a < Q; ++a) r[a] += v[a];
  if (is_wall[i]) {
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const int b = opp(a);
      if (b > a) {
        const real m = (real)0.5 * (r[a] + r[b]);
        r[a] = m;
        r[b] = m;
      }
    }
  }
  store_set(ps, i, Np, r);
  if (comp) {
    double sh = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) sh += (double)r[a];
    cs.r[i] = (cs.Cn[i] + rc) - sh;
  }
}

// init: psi_bar^0 = psi_eq(C, u, p), then the wall operator
template <typename real>
__global__ void __launch_bounds__(BLOCK) k3_init(int N, int Np, StepParams P, const double* __restrict__ C,
                                                const double* __restrict__ U, const double* __restrict__ Pr,
                                                const uint8_t* __restrict__ is_wall, real* __restrict__ pop,
                                                double* __restrict__ rC) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= N) return;
  const double c = C[i], ux = U[3 * i], uy = U[3 * i + 1], uz = U[3 * i + 2], p = Pr[i];
  const double rho = c * P.rho_l + (1.0 - c) * P.rho_v, uu = ux * ux + uy * uy + uz * uz;
  double s[NPOP];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy + ez(a) * uz;
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
  real gv[Q], hv[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    gv[a] = (real)s[a];
    hv[a] = (real)s[Q + a];
  }
  store_set(pop, i, Np, gv);
  store_set(pop + (size_t)QS * Np, i, Np, hv);
  if (rC) {  // FP32: the remainder makes C exactly the given composition
    double sh = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) sh += (double)(real)s[Q + a];
    rC[i] = c - sh;
  }
}

}  // namespace felbm3d
