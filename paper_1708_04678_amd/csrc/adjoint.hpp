// Reverse-mode (vector-Jacobian) kernels of one FE-LBM step, the transpose of
// the forward sequence in kernels.hpp.  Given lam = dL/dpsi_bar^{n+1} they
// produce dL/dpsi_bar^n and add dL/dOmega_c (wetting potential of each wall
// node) to a running gradient.  The forward fields of step n (C, p, u, mu,
// element gradients, Laplacians) are recomputed from psi_bar^n beforehand by
// the forward field kernels.  Every output is gathered by one thread (no
// atomics); the adjoint arithmetic runs in double, lam is stored in real.
//
// Forward map of a step (FP64 semantics):
//   C = sum h, p = sum g, rho = rho_v + C (rho_l - rho_v), u = 3 sum e g / rho
//   psi_hat = psi - omega(C) (psi - psi_eq(C, p, rho, u))
//   b_{a,i} = sum_{T ni i} A_T (dt/3 + dt^2/2 e_a.grad N_i) q_{a,T},
//   q_{a,T} = Phi_{a,T}(Cbar, ubar, mubar, grad C, grad p, lap mu) - e_a . sum_v psi_hat_{a,v} grad N_v
//   x = P b (K Chebyshev-step Richardson sweeps), psi^{n+1} = W (psi_hat + x)
#pragma once

#include "kernels.hpp"

namespace felbm {

struct AdjGeom {
  const int* tri;       // [3][E]
  const int* enbr;      // [3][E]
  const int* erev;      // [3][E] local edge index of this element inside its neighbour
  const double* geo;    // [7][E]
  const int* n2e_ptr;   // [N+1]
  const int* n2e;       // element*4 + local vertex
  const double* mass;   // [N] lumped mass (patch volume = 3 m)
  const int* wall_nbr;  // [2][N]
  const double* wall_len;
  const double* bc;     // [N] phi_c / kappa
  const uint8_t* is_wall;
  int N, Np, E;
};

// element adjoint record, [9][E] double
enum { EA_C = 0, EA_UX, EA_UY, EA_MU, EA_GCX, EA_GCY, EA_GPX, EA_GPY, EA_LM, EA_N };

// A1: f = (W lam) / m, the right-hand side of the transposed solve
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_adj_prep(AdjGeom g, const real* __restrict__ lam, real* __restrict__ f) {
  const int i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= g.N) return;
  double l[NPOP];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) l[a] = (double)lam[a * g.Np + i];
  if (g.is_wall[i]) {
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const int b = opp(a);
      if (b > a) {
        const double mg = 0.5 * (l[a] + l[b]), mh = 0.5 * (l[Q + a] + l[Q + b]);
        l[a] = mg; l[b] = mg; l[Q + a] = mh; l[Q + b] = mh;
      }
    }
  }
  const double im = 1.0 / g.mass[i];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) f[a * g.Np + i] = (real)(l[a] * im);
}

// lam_q_{a,T} = A_T sum_{t} (dt/3 + dt^2/2 e_a.grad N_t) lam_b_{a,v_t}
template <typename real>
__device__ __forceinline__ void adj_lamq(const AdjGeom& g, int e, const real* __restrict__ lb, double dt,
                                         double (&lq)[NPOP]) {
  const int v0 = g.tri[e], v1 = g.tri[g.E + e], v2 = g.tri[2 * g.E + e];
  const double A = g.geo[e];
  double gx[3], gy[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    gx[t] = g.geo[(1 + 2 * t) * g.E + e];
    gy[t] = g.geo[(2 + 2 * t) * g.E + e];
  }
  const double c1 = dt / 3.0, c2 = 0.5 * dt * dt;
#pragma unroll
  for (int p = 0; p < NPOP; ++p) {
    const int a = p % Q;
    const double en0 = ex(a) * gx[0] + ey(a) * gy[0], en1 = ex(a) * gx[1] + ey(a) * gy[1];
    const double en2 = ex(a) * gx[2] + ey(a) * gy[2];
    lq[p] = A * ((c1 + c2 * en0) * (double)lb[p * g.Np + v0] + (c1 + c2 * en1) * (double)lb[p * g.Np + v1] +
                 (c1 + c2 * en2) * (double)lb[p * g.Np + v2]);
  }
}

// A3: per element, the transpose of the P0 forces eq:G / eq:H at barycentric
// values, fed by lam_Phi = lam_q.  Writes the element adjoint record and
// lam_q itself ([NPOP][E], in the compute precision) for the streaming
// transpose.
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_adj_force(AdjGeom g, StepParams P, const real* __restrict__ lb,
                                                    const double* __restrict__ Cn, const real* __restrict__ uxn,
                                                    const real* __restrict__ uyn, const double* __restrict__ mu,
                                                    const double* __restrict__ gC, const real* __restrict__ gp,
                                                    const double* __restrict__ lapmu, double* __restrict__ ea,
                                                    real* __restrict__ lqe) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= g.E) return;
  double lq[NPOP];
  adj_lamq(g, e, lb, P.dt, lq);
#pragma unroll
  for (int p = 0; p < NPOP; ++p) lqe[p * g.E + e] = (real)lq[p];
  const int v0 = g.tri[e], v1 = g.tri[g.E + e], v2 = g.tri[2 * g.E + e];
  const double Cb = (Cn[v0] + Cn[v1] + Cn[v2]) * (1.0 / 3.0);
  const double mub = (mu[v0] + mu[v1] + mu[v2]) * (1.0 / 3.0);
  const double ux = ((double)uxn[v0] + (double)uxn[v1] + (double)uxn[v2]) * (1.0 / 3.0);
  const double uy = ((double)uyn[v0] + (double)uyn[v1] + (double)uyn[v2]) * (1.0 / 3.0);
  const double drho = P.rho_l - P.rho_v, rhob = P.rho_v + Cb * drho;
  const double gcx = gC[e], gcy = gC[g.E + e], gpx = (double)gp[e], gpy = (double)gp[g.E + e];
  const double cr = CS2 * drho;
  const double ax = cr * gcx, ay = cr * gcy;            // c_s^2 grad rho
  const double bx = mub * gcx, by = mub * gcy;          // mu grad C
  const double coef = Cb / (rhob * CS2);
  const double Xx = gcx - coef * (gpx - bx), Xy = gcy - coef * (gpy - by);
  const double d = P.mobility * lapmu[e];
  const double uu = ux * ux + uy * uy;
  double lax = 0, lay = 0, lbx = 0, lby = 0, lXx = 0, lXy = 0, ld = 0, lux = 0, luy = 0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double exa = ex(a), eya = ey(a), w = wq(a);
    const double eu = exa * ux + eya * uy;
    const double G = w * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    const double dGx = w * (3.0 * exa + 9.0 * eu * exa - 3.0 * ux), dGy = w * (3.0 * eya + 9.0 * eu * eya - 3.0 * uy);
    const double mx = exa - ux, my = eya - uy;          // e - u
    const double sa = mx * ax + my * ay, sb = mx * bx + my * by, sX = mx * Xx + my * Xy;
    const double dg = lq[a], dh = lq[Q + a];
    // Phi_g = sa (G - w) + sb G ;  Phi_h = (sX + d) G
    lax += dg * (G - w) * mx; lay += dg * (G - w) * my;
    lbx += dg * G * mx;       lby += dg * G * my;
    lXx += dh * G * mx;       lXy += dh * G * my;
    ld += dh * G;
    const double lG = dg * (sa + sb) + dh * (sX + d);
    lux += lG * dGx - dg * ((G - w) * ax + G * bx) - dh * G * Xx;
    luy += lG * dGy - dg * ((G - w) * ay + G * by) - dh * G * Xy;
  }
  // back through a = cr gC, b = mu gC, X = gC (1 + coef mu) - coef gp, d = M lap mu
  double lgcx = cr * lax + mub * lbx + (1.0 + coef * mub) * lXx;
  double lgcy = cr * lay + mub * lby + (1.0 + coef * mub) * lXy;
  const double lgpx = -coef * lXx, lgpy = -coef * lXy;
  const double lcoef = -(lXx * (gpx - bx) + lXy * (gpy - by));
  const double lmub = lbx * gcx + lby * gcy + coef * (lXx * gcx + lXy * gcy);
  const double lCb = lcoef * P.rho_v / (rhob * rhob * CS2);   // d(C/rho)/dC = rho_v / rho^2
  const int E = g.E;
  ea[EA_C * E + e] = lCb;
  ea[EA_UX * E + e] = lux;
  ea[EA_UY * E + e] = luy;
  ea[EA_MU * E + e] = lmub;
  ea[EA_GCX * E + e] = lgcx;
  ea[EA_GCY * E + e] = lgcy;
  ea[EA_GPX * E + e] = lgpx;
  ea[EA_GPY * E + e] = lgpy;
  ea[EA_LM * E + e] = P.mobility * ld;
}

// A4: per node, lam_hat = W lam - sum_{T ni v} lam_q_{a,T} e_a.grad N_v, with lam_q
// as stored by k_adj_force
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_adj_stream(AdjGeom g, const real* __restrict__ lam,
                                                     const real* __restrict__ lqe, real* __restrict__ lhat) {
  const int v = xcd_block() * BLOCK + threadIdx.x;
  if (v >= g.N) return;
  double l[NPOP];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) l[a] = (double)lam[a * g.Np + v];
  if (g.is_wall[v]) {
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const int b = opp(a);
      if (b > a) {
        const double mg = 0.5 * (l[a] + l[b]), mh = 0.5 * (l[Q + a] + l[Q + b]);
        l[a] = mg; l[b] = mg; l[Q + a] = mh; l[Q + b] = mh;
      }
    }
  }
  for (int q = g.n2e_ptr[v]; q < g.n2e_ptr[v + 1]; ++q) {
    const int packed = g.n2e[q];
    const int e = packed >> 2, lv = packed & 3;
    const double gx = g.geo[(1 + 2 * lv) * g.E + e], gy = g.geo[(2 + 2 * lv) * g.E + e];
#pragma unroll
    for (int p = 0; p < NPOP; ++p) {
      const int a = p % Q;
      l[p] -= (double)lqe[p * g.E + e] * (ex(a) * gx + ey(a) * gy);
    }
  }
#pragma unroll
  for (int a = 0; a < NPOP; ++a) lhat[a * g.Np + v] = (real)l[a];
}

// A5: per element, lam_gmu = transpose of lap mu_T = -sum_{v: T'_v} grad N_v . (g_T + g_T'_v)
__global__ void __launch_bounds__(BLOCK) k_adj_gmu(AdjGeom g, const double* __restrict__ ea,
                                                  double* __restrict__ lgmu) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= g.E) return;
  const int E = g.E;
  const double lm = ea[EA_LM * E + e];
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int nb = g.enbr[l * E + e];
    if (nb < 0) continue;
    sx -= lm * g.geo[(1 + 2 * l) * E + e];
    sy -= lm * g.geo[(2 + 2 * l) * E + e];
    const int lr = g.erev[l * E + e];
    const double lmn = ea[EA_LM * E + nb];
    sx -= lmn * g.geo[(1 + 2 * lr) * E + nb];
    sy -= lmn * g.geo[(2 + 2 * lr) * E + nb];
  }
  lgmu[e] = sx;
  lgmu[E + e] = sy;
}

// A6: per node, lam_mu = sum_{T ni v} (lam_mubar_T / 3 + lam_gmu_T . grad N_v)
__global__ void __launch_bounds__(BLOCK) k_adj_mu(AdjGeom g, const double* __restrict__ ea,
                                                 const double* __restrict__ lgmu, double* __restrict__ lmu) {
  const int v = xcd_block() * BLOCK + threadIdx.x;
  if (v >= g.N) return;
  const int E = g.E;
  double s = 0.0;
  for (int q = g.n2e_ptr[v]; q < g.n2e_ptr[v + 1]; ++q) {
    const int packed = g.n2e[q];
    const int e = packed >> 2, l = packed & 3;
    s += ea[EA_MU * E + e] * (1.0 / 3.0) + lgmu[e] * g.geo[(1 + 2 * l) * E + e] +
         lgmu[E + e] * g.geo[(2 + 2 * l) * E + e];
  }
  lmu[v] = s;
}

// A7: per element, lam_gC = force part + transpose of the patch Laplacian:
// lap C_k gets -A_T grad N_l . (g_T + g_T') / V_k from each patch element T
// whose edge opposite k is interior (V_k = 3 m_k), lam_lapC_k = -kappa lam_mu_k
__global__ void __launch_bounds__(BLOCK) k_adj_gC(AdjGeom g, StepParams P, const double* __restrict__ ea,
                                                 const double* __restrict__ lmu, double* __restrict__ lgC) {
  const int e = xcd_block() * BLOCK + threadIdx.x;
  if (e >= g.E) return;
  const int E = g.E;
  double sx = ea[EA_GCX * E + e], sy = ea[EA_GCY * E + e];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const int nb = g.enbr[l * E + e];
    if (nb < 0) continue;
    const int k = g.tri[l * E + e];
    const double wk = -P.kappa * lmu[k] / (3.0 * g.mass[k]) * (-g.geo[e]);
    sx += wk * g.geo[(1 + 2 * l) * E + e];
    sy += wk * g.geo[(2 + 2 * l) * E + e];
    const int lr = g.erev[l * E + e];
    const int kn = g.tri[lr * E + nb];
    const double wn = -P.kappa * lmu[kn] / (3.0 * g.mass[kn]) * (-g.geo[nb]);
    sx += wn * g.geo[(1 + 2 * lr) * E + nb];
    sy += wn * g.geo[(2 + 2 * lr) * E + nb];
  }
  lgC[e] = sx;
  lgC[E + e] = sy;
}

// partial derivatives of the wall flux F(Ca, Cb, ra, rb, len) (see wall_flux)
__device__ __forceinline__ void wall_flux_d(double Ca, double Cb, double ra, double rb, double len, double& dCa,
                                            double& dCb, double& dra, double& drb) {
  const double Cm = 0.5 * (Ca + Cb), rm = 0.5 * (ra + rb);
  const double s = -len * (1.0 / 6.0);
  const double fm = Cm - Cm * Cm, dfm = 1.0 - 2.0 * Cm;
  dCa = s * (ra * (1.0 - 2.0 * Ca) + 2.0 * rm * dfm);
  dCb = s * (rb * (1.0 - 2.0 * Cb) + 2.0 * rm * dfm);
  dra = s * ((Ca - Ca * Ca) + 2.0 * fm);
  drb = s * ((Cb - Cb * Cb) + 2.0 * fm);
}

// A8: per node, all remaining transposes: element-gathered parts of lam_C,
// lam_p, lam_u; the bulk term of mu; the wetting fluxes (including dL/dphi);
// the collision and the moments.  Overwrites lam with dL/dpsi_bar^n and adds
// dL/dOmega_c into gomega.
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_adj_node(AdjGeom g, StepParams P, double bc_scale,
                                                   const real* __restrict__ pop, const double* __restrict__ Cn,
                                                   const real* __restrict__ pn, const real* __restrict__ uxn,
                                                   const real* __restrict__ uyn, const double* __restrict__ ea,
                                                   const double* __restrict__ lgC, const double* __restrict__ lmu,
                                                   const real* __restrict__ lhat, real* __restrict__ lam,
                                                   double* __restrict__ gomega) {
  const int v = xcd_block() * BLOCK + threadIdx.x;
  if (v >= g.N) return;
  const int E = g.E;
  const double C = Cn[v];
  double lC = 0.0, lp = 0.0, lux = 0.0, luy = 0.0, lbc = 0.0;
  // element-gathered contributions
  for (int q = g.n2e_ptr[v]; q < g.n2e_ptr[v + 1]; ++q) {
    const int packed = g.n2e[q];
    const int e = packed >> 2, l = packed & 3;
    const double gx = g.geo[(1 + 2 * l) * E + e], gy = g.geo[(2 + 2 * l) * E + e];
    lC += ea[EA_C * E + e] * (1.0 / 3.0) + lgC[e] * gx + lgC[E + e] * gy;
    lp += ea[EA_GPX * E + e] * gx + ea[EA_GPY * E + e] * gy;
    lux += ea[EA_UX * E + e] * (1.0 / 3.0);
    luy += ea[EA_UY * E + e] * (1.0 / 3.0);
    // wall edges opposite the other two vertices k that contain v (their lap C)
#pragma unroll
    for (int t = 1; t < 3; ++t) {
      const int lk = (l + t) % 3;
      if (g.enbr[lk * E + e] >= 0) continue;
      const int k = g.tri[lk * E + e];
      const int a = g.tri[((lk + 1) % 3) * E + e], b = g.tri[((lk + 2) % 3) * E + e];
      const double gkx = g.geo[(1 + 2 * lk) * E + e], gky = g.geo[(2 + 2 * lk) * E + e];
      const double len = 2.0 * g.geo[e] * sqrt(gkx * gkx + gky * gky);
      double dCa, dCb, dra, drb;
      wall_flux_d(Cn[a], Cn[b], g.bc[a], g.bc[b], len, dCa, dCb, dra, drb);
      const double llk = -P.kappa * lmu[k] / (3.0 * g.mass[k]);
      lC += llk * (a == v ? dCa : dCb);
      lbc += llk * (a == v ? dra : drb);
    }
  }
  // bulk part of mu and the wall edges incident to v (own lap C and the neighbour's)
  const double lmv = lmu[v];
  lC += lmv * 2.0 * P.beta * (6.0 * C * C - 6.0 * C + 1.0);
  const double llv = -P.kappa * lmv / (3.0 * g.mass[v]);
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int j = g.wall_nbr[w * g.N + v];
    if (j < 0) continue;
    const double len = g.wall_len[w * g.N + v];
    double dCa, dCb, dra, drb;
    wall_flux_d(C, Cn[j], g.bc[v], g.bc[j], len, dCa, dCb, dra, drb);
    const double llj = -P.kappa * lmu[j] / (3.0 * g.mass[j]);
    lC += llv * dCa + llj * dCa;  // F(C_v, C_j) enters lap C_v and, with the same value, lap C_j
    lbc += llv * dra + llj * dra;
  }
  if (g.is_wall[v]) gomega[v] += lbc * bc_scale;
  // collision (eqn::collide) and moments
  double ps[NPOP], lh[NPOP];
#pragma unroll
  for (int a = 0; a < NPOP; ++a) {
    ps[a] = (double)pop[a * g.Np + v];
    lh[a] = (double)lhat[a * g.Np + v];
  }
  const double p = (double)pn[v], ux = (double)uxn[v], uy = (double)uyn[v];
  const double drho = P.rho_l - P.rho_v, rho = P.rho_v + C * drho;
  const double s = C * P.inv_tau_l + (1.0 - C) * P.inv_tau_v;
  const double om = 1.0 / (1.0 / s + 0.5);
  const double uu = ux * ux + uy * uy;
  double lom = 0.0, lrho = 0.0;
  double out[NPOP];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double exa = ex(a), eya = ey(a), w = wq(a);
    const double eu = exa * ux + eya * uy;
    const double Pa = eu + 1.5 * eu * eu - 0.5 * uu;
    const double geq = w * (p + rho * Pa), heq = w * C * (1.0 + 3.0 * Pa);
    lom -= lh[a] * (ps[a] - geq) + lh[Q + a] * (ps[Q + a] - heq);
    out[a] = (1.0 - om) * lh[a];
    out[Q + a] = (1.0 - om) * lh[Q + a];
    const double lg = om * lh[a], lhq = om * lh[Q + a];
    lp += w * lg;
    lrho += w * Pa * lg;
    lC += w * (1.0 + 3.0 * Pa) * lhq;
    const double lP = w * (rho * lg + 3.0 * C * lhq);
    lux += lP * (exa + 3.0 * eu * exa - ux);
    luy += lP * (eya + 3.0 * eu * eya - uy);
  }
  const double dom = 1.0 / ((1.0 + 0.5 * s) * (1.0 + 0.5 * s));
  lC += lom * dom * (P.inv_tau_l - P.inv_tau_v);
  // u = 3 j / rho, rho = rho_v + C (rho_l - rho_v)
  const double ljx = 3.0 * lux / rho, ljy = 3.0 * luy / rho;
  lrho -= (ux * lux + uy * luy) / rho;
  lC += drho * lrho;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    lam[a * g.Np + v] = (real)(out[a] + lp + ex(a) * ljx + ey(a) * ljy);
    lam[(Q + a) * g.Np + v] = (real)(out[Q + a] + lC);
  }
}

// lam^{N_steps}: dL/dpsi_bar from dL/dC (C = sum h), read in caller node order
template <typename real>
__global__ void __launch_bounds__(BLOCK) k_adj_init(int N, int Np, const int* __restrict__ node_perm,
                                                   const double* __restrict__ dLdC, real* __restrict__ lam) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= N) return;
  const real v = (real)dLdC[node_perm[k]];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    lam[a * Np + k] = (real)0;
    lam[(Q + a) * Np + k] = v;
  }
}

// internal -> caller node order
__global__ void __launch_bounds__(BLOCK) k_to_caller(int N, const int* __restrict__ node_perm,
                                                    const double* __restrict__ src, double* __restrict__ dst) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k < N) dst[node_perm[k]] = src[k];
}

}  // namespace felbm
