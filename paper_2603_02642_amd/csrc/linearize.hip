// Constraint-data formation on the device (supplementary section I, step a0).
//
// Kernel 1, one workgroup per instance: nonlinear forward-Euler rollout of the
// nominal controls (thread 0) and the analytic Jacobians A_k, B_k (threads in
// parallel over k).
// Kernel 2, one thread per constraint: the gradient w of the constraint at
// x_t and its value g0, then the adjoint recursion
//   lambda_t = w,  b_{j,i} = B_i' lambda_{i+1},  lambda_i = A_i' lambda_{i+1},
//   b_hat_j[i] = r lambda_i   (i = t-1 .. 0; block t holds r w and b = 0),
// written into the compact cone layout (float64 and float32 copies).
// Control bounds s u_{k,i} <= s bound give b = s e_i in block k and b_hat = 0.
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace nrto {

constexpr double GRAV = 9.81;

template <int NX, int NU>
__device__ void xdot_dev(int dyn, const double* prm, const ParamOffsets& po, double mass, const double* x,
                         const double* u, double* f) {
  if (dyn == NRTO_DYN_UNICYCLE) {
    f[0] = u[0] * cos(x[2]);
    f[1] = u[0] * sin(x[2]);
    f[2] = u[1];
  } else if (dyn == NRTO_DYN_QUADROTOR) {
    const double ph = x[6], th = x[7], ps = x[8];
    const double cph = cos(ph), sph = sin(ph), cth = cos(th), sth = sin(th), cps = cos(ps), sps = sin(ps);
    const double J1 = prm[po.inertia], J2 = prm[po.inertia + 1], J3 = prm[po.inertia + 2];
    const double p = x[9], q = x[10], r = x[11];
    f[0] = x[3];
    f[1] = x[4];
    f[2] = x[5];
    const double fm = u[0] / mass;
    f[3] = fm * (cps * sth * cph + sps * sph);
    f[4] = fm * (sps * sth * cph - cps * sph);
    f[5] = fm * (cth * cph) - GRAV;
    const double tth = sth / cth;
    f[6] = p + sph * tth * q + cph * tth * r;
    f[7] = cph * q - sph * r;
    f[8] = (sph * q + cph * r) / cth;
    f[9] = (u[1] - (J3 - J2) * q * r) / J1;
    f[10] = (u[2] - (J1 - J3) * p * r) / J2;
    f[11] = (u[3] - (J2 - J1) * p * q) / J3;
  } else {
    for (int i = 0; i < 7; ++i) {
      f[i] = x[7 + i];
      f[7 + i] = u[i];
    }
  }
}

// Continuous-time Jacobians fx (NX x NX), fu (NX x NU), row-major.
template <int NX, int NU>
__device__ void jac_dev(int dyn, const double* prm, const ParamOffsets& po, double mass, const double* x,
                        const double* u, double* fx, double* fu) {
  for (int i = 0; i < NX * NX; ++i) fx[i] = 0.0;
  for (int i = 0; i < NX * NU; ++i) fu[i] = 0.0;
  if (dyn == NRTO_DYN_UNICYCLE) {
    const double c = cos(x[2]), s = sin(x[2]);
    fx[0 * NX + 2] = -u[0] * s;
    fx[1 * NX + 2] = u[0] * c;
    fu[0 * NU + 0] = c;
    fu[1 * NU + 0] = s;
    fu[2 * NU + 1] = 1.0;
  } else if (dyn == NRTO_DYN_QUADROTOR) {
    const double ph = x[6], th = x[7], ps = x[8];
    const double cph = cos(ph), sph = sin(ph), cth = cos(th), sth = sin(th), cps = cos(ps), sps = sin(ps);
    const double J1 = prm[po.inertia], J2 = prm[po.inertia + 1], J3 = prm[po.inertia + 2];
    const double p = x[9], q = x[10], r = x[11];
    const double fm = u[0] / mass;
    fx[0 * NX + 3] = fx[1 * NX + 4] = fx[2 * NX + 5] = 1.0;
    // d(R e3)/d(phi, theta, psi)
    fx[3 * NX + 6] = fm * (sps * cph - cps * sth * sph);
    fx[3 * NX + 7] = fm * (cps * cth * cph);
    fx[3 * NX + 8] = fm * (cps * sph - sps * sth * cph);
    fx[4 * NX + 6] = fm * (-cps * cph - sps * sth * sph);
    fx[4 * NX + 7] = fm * (sps * cth * cph);
    fx[4 * NX + 8] = fm * (sps * sph + cps * sth * cph);
    fx[5 * NX + 6] = -fm * cth * sph;
    fx[5 * NX + 7] = -fm * sth * cph;
    fu[3 * NU + 0] = (cps * sth * cph + sps * sph) / mass;
    fu[4 * NU + 0] = (sps * sth * cph - cps * sph) / mass;
    fu[5 * NU + 0] = (cth * cph) / mass;
    const double tth = sth / cth, sec2 = 1.0 / (cth * cth);
    fx[6 * NX + 6] = cph * tth * q - sph * tth * r;
    fx[6 * NX + 7] = (sph * q + cph * r) * sec2;
    fx[6 * NX + 9] = 1.0;
    fx[6 * NX + 10] = sph * tth;
    fx[6 * NX + 11] = cph * tth;
    fx[7 * NX + 6] = -sph * q - cph * r;
    fx[7 * NX + 10] = cph;
    fx[7 * NX + 11] = -sph;
    fx[8 * NX + 6] = (cph * q - sph * r) / cth;
    fx[8 * NX + 7] = (sph * q + cph * r) * sth * sec2;
    fx[8 * NX + 10] = sph / cth;
    fx[8 * NX + 11] = cph / cth;
    fx[9 * NX + 10] = -(J3 - J2) * r / J1;
    fx[9 * NX + 11] = -(J3 - J2) * q / J1;
    fx[10 * NX + 9] = -(J1 - J3) * r / J2;
    fx[10 * NX + 11] = -(J1 - J3) * p / J2;
    fx[11 * NX + 9] = -(J2 - J1) * q / J3;
    fx[11 * NX + 10] = -(J2 - J1) * p / J3;
    fu[9 * NU + 1] = 1.0 / J1;
    fu[10 * NU + 2] = 1.0 / J2;
    fu[11 * NU + 3] = 1.0 / J3;
  } else {
    for (int i = 0; i < 7; ++i) {
      fx[i * NX + 7 + i] = 1.0;
      fu[(7 + i) * NU + i] = 1.0;
    }
  }
}

// Standard-DH frame origins o_1..o_7 and the 3x7 position Jacobian of origin
// `pt` (0-based, frame pt+1) for joint angles q: revolute joint m moves it by
// z_m x (o_{pt+1} - o_m).
__device__ void arm_point(const double* links, const double* q, int pt, double* pos, double* J) {
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double o[3] = {0, 0, 0};
  double Z[8][3], O[8][3];
  Z[0][0] = 0; Z[0][1] = 0; Z[0][2] = 1;
  O[0][0] = O[0][1] = O[0][2] = 0;
  for (int i = 0; i < 7; ++i) {
    const double al = (i == 6) ? 0.0 : ((i % 2 == 0) ? M_PI / 2 : -M_PI / 2);
    const double ct = cos(q[i]), st = sin(q[i]), ca = cos(al), sa = sin(al);
    const double a = links[i];
    // A_i = Rz(q) Tz(0) Tx(a) Rx(al)
    const double Ar[9] = {ct, -st * ca, st * sa, st, ct * ca, -ct * sa, 0.0, sa, ca};
    const double At[3] = {a * ct, a * st, 0.0};
    double Rn[9];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) Rn[r * 3 + cc] = R[r * 3] * Ar[cc] + R[r * 3 + 1] * Ar[3 + cc] + R[r * 3 + 2] * Ar[6 + cc];
    double on[3];
    for (int r = 0; r < 3; ++r) on[r] = o[r] + R[r * 3] * At[0] + R[r * 3 + 1] * At[1] + R[r * 3 + 2] * At[2];
    for (int r = 0; r < 9; ++r) R[r] = Rn[r];
    for (int r = 0; r < 3; ++r) o[r] = on[r];
    for (int r = 0; r < 3; ++r) {
      O[i + 1][r] = o[r];
      Z[i + 1][r] = R[r * 3 + 2];
    }
  }
  for (int r = 0; r < 3; ++r) pos[r] = O[pt + 1][r];
  for (int m = 0; m < 7; ++m) {
    double d[3] = {0, 0, 0};
    if (m <= pt)
      for (int r = 0; r < 3; ++r) d[r] = O[pt + 1][r] - O[m][r];
    J[0 * 7 + m] = Z[m][1] * d[2] - Z[m][2] * d[1];
    J[1 * 7 + m] = Z[m][2] * d[0] - Z[m][0] * d[2];
    J[2 * 7 + m] = Z[m][0] * d[1] - Z[m][1] * d[0];
  }
}

template <int NX, int NU>
__device__ void rollout_and_jac(const DevPtrs& g, int ii) {
  const InstDev& d = g.inst[ii];
  const int T = d.T;
  const double* prm = g.prm + d.oP;
  const ParamOffsets po = param_offsets(NX, NU, d.n_obs);
  double* xh = g.xhat + d.oX;
  const double* uh = g.uhat + d.oU;
  if (threadIdx.x == 0) {
    double x[NX], f[NX];
    for (int i = 0; i < NX; ++i) x[i] = prm[po.x0 + i];
    for (int i = 0; i < NX; ++i) xh[i] = x[i];
    for (int k = 0; k < T; ++k) {
      xdot_dev<NX, NU>(d.dyn, prm, po, d.mass, x, uh + k * NU, f);
      for (int i = 0; i < NX; ++i) x[i] += d.dt * f[i];
      for (int i = 0; i < NX; ++i) xh[(k + 1) * NX + i] = x[i];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < T; k += blockDim.x) {
    double fx[NX * NX], fu[NX * NU];
    jac_dev<NX, NU>(d.dyn, prm, po, d.mass, xh + k * NX, uh + k * NU, fx, fu);
    double* A = g.A + d.oA + (int64_t)k * NX * NX;
    double* B = g.B + d.oB + (int64_t)k * NX * NU;
    for (int i = 0; i < NX; ++i)
      for (int j = 0; j < NX; ++j) A[i * NX + j] = (i == j ? 1.0 : 0.0) + d.dt * fx[i * NX + j];
    for (int i = 0; i < NX * NU; ++i) B[i] = d.dt * fu[i];
  }
}

__global__ void rollout_kernel(DevPtrs g) {
  const int ii = blockIdx.x;
  const int nx = g.inst[ii].nx;
  if (nx == 3) rollout_and_jac<3, 2>(g, ii);
  else if (nx == 12) rollout_and_jac<12, 4>(g, ii);
  else rollout_and_jac<14, 7>(g, ii);
}

// Value and state gradient of state constraint j (time slice entry) at x_t.
template <int NX, int NU>
__device__ double state_cons_eval(const DevPtrs& g, const InstDev& d, int j, const int32_t* m, const double* xt,
                                  double* w) {
  const double* prm = g.prm + d.oP;
  const ParamOffsets po = param_offsets(NX, NU, d.n_obs);
  for (int l = 0; l < NX; ++l) w[l] = 0.0;
  const int npts = (d.dyn == NRTO_DYN_ARM) ? 7 : 1;
  const int t = m[CM_TIME];
  const int32_t* tls = g.tl + d.oTL;
  const int jj = j - tls[t];
  double gv;
  if (jj < d.n_obs * npts) {
    const int o = jj / npts, pt = jj - o * npts;
    const double* ob = prm + po.obs + 4 * o;
    double pos[3] = {0, 0, 0};
    double J[3 * 7];
    int pd;
    if (d.dyn == NRTO_DYN_ARM) {
      arm_point(prm + po.links, xt, pt, pos, J);
      pd = 3;
    } else {
      pd = (d.dyn == NRTO_DYN_UNICYCLE) ? 2 : 3;
      for (int a = 0; a < pd; ++a) pos[a] = xt[a];
    }
    double dv[3] = {0, 0, 0};
    double nd2 = 0.0;
    for (int a = 0; a < pd; ++a) {
      dv[a] = pos[a] - ob[a];
      nd2 += dv[a] * dv[a];
    }
    const double nd = sqrt(nd2);
    double dir[3] = {0, 0, 0};
    if (nd > 0.0) {
      for (int a = 0; a < pd; ++a) dir[a] = dv[a] / nd;
    } else {
      dir[0] = 1.0;
    }
    gv = ob[3] - nd;
    if (d.dyn == NRTO_DYN_ARM) {
      for (int q = 0; q < 7; ++q) w[q] = -(J[q] * dir[0] + J[7 + q] * dir[1] + J[14 + q] * dir[2]);
    } else {
      for (int a = 0; a < pd; ++a) w[a] = -dir[a];
    }
  } else {
    const int i = m[CM_CIDX], s = m[CM_CSIGN];
    if (s > 0) {
      gv = xt[i] - prm[po.xhi + i];
      w[i] = 1.0;
    } else {
      gv = prm[po.xlo + i] - xt[i];
      w[i] = -1.0;
    }
  }
  return gv;
}

template <int NX, int NU>
__device__ void cone_data(const DevPtrs& g, const InstDev& d, int j) {
  const int32_t* m = g.cmeta + (d.cone0 + j) * CM_N;
  const double* prm = g.prm + d.oP;
  const ParamOffsets po = param_offsets(NX, NU, d.n_obs);
  const double* xh = g.xhat + d.oX;
  const double* uh = g.uhat + d.oU;
  const int e0 = m[CM_EOFF], nb = m[CM_NBLK], bo = m[CM_BOFF];
  double* bh = g.bhat64 + d.ent0 + e0;
  float* bh32 = g.bhat32 + d.ent0 + e0;
  double* bv = g.bvec64 + d.bv0 + (int64_t)bo * NU;
  float* bv32 = g.bvec32 + d.bv0 + (int64_t)bo * NU;
  double* wout = g.w + d.oW + (int64_t)j * NX;
  double* g0 = g.carr + (int64_t)CA_G0 * g.ncones + d.cone0 + j;
  const double r = d.radius;
  bh[0] = 0.0;
  bh32[0] = 0.0f;
  if (m[CM_KIND] == 1) {
    const int k = m[CM_TIME], i = m[CM_CIDX], s = m[CM_CSIGN];
    const double bound = (s > 0) ? prm[po.uhi + i] : prm[po.ulo + i];
    *g0 = s * uh[k * NU + i] - s * bound;
    for (int l = 0; l < NX; ++l) {
      bh[1 + l] = 0.0;
      bh32[1 + l] = 0.0f;
      wout[l] = 0.0;
    }
    for (int u = 0; u < NU; ++u) {
      bv[u] = (u == i) ? (double)s : 0.0;
      bv32[u] = (float)bv[u];
    }
    return;
  }
  const int t = m[CM_TIME];
  const double* xt = xh + t * NX;
  double w[NX];
  const double gv = state_cons_eval<NX, NU>(g, d, j, m, xt, w);
  (void)po;
  *g0 = gv;
  for (int l = 0; l < NX; ++l) wout[l] = w[l];
  // adjoint recursion; block t first (b = 0)
  double lam[NX];
  for (int l = 0; l < NX; ++l) lam[l] = w[l];
  for (int l = 0; l < NX; ++l) {
    bh[1 + t * NX + l] = r * lam[l];
    bh32[1 + t * NX + l] = (float)(r * lam[l]);
  }
  for (int u = 0; u < NU; ++u) {
    bv[t * NU + u] = 0.0;
    bv32[t * NU + u] = 0.0f;
  }
  for (int i = t - 1; i >= 0; --i) {
    const double* A = g.A + d.oA + (int64_t)i * NX * NX;
    const double* B = g.B + d.oB + (int64_t)i * NX * NU;
    for (int u = 0; u < NU; ++u) {
      double s = 0.0;
      for (int l = 0; l < NX; ++l) s += B[l * NU + u] * lam[l];
      bv[i * NU + u] = s;
      bv32[i * NU + u] = (float)s;
    }
    double nl[NX];
    for (int a = 0; a < NX; ++a) {
      double s = 0.0;
      for (int l = 0; l < NX; ++l) s += A[l * NX + a] * lam[l];
      nl[a] = s;
    }
    for (int l = 0; l < NX; ++l) {
      lam[l] = nl[l];
      bh[1 + i * NX + l] = r * lam[l];
      bh32[1 + i * NX + l] = (float)(r * lam[l]);
    }
  }
  (void)nb;
}

__global__ void cone_data_kernel(DevPtrs g, int n_inst) {
  const int ii = blockIdx.y;
  const InstDev& d = g.inst[ii];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.ng; j += gridDim.x * blockDim.x) {
    if (d.nx == 3) cone_data<3, 2>(g, d, j);
    else if (d.nx == 12) cone_data<12, 4>(g, d, j);
    else cone_data<14, 7>(g, d, j);
  }
}

// Trust-region test of one successive-linearisation step (see the oracle's scp
// module for the merit definitions).  A step whose SOCP solve did not reach its
// tolerance is rejected (the radius shrinks).  One workgroup per instance; out[4*ii..]
// receives (accepted, merit_cur, merit_act, merit_pred).
template <int NX, int NU>
__device__ void scp_eval(const DevPtrs& g, int ii, double w_p, double* out) {
  InstDev& d = g.inst[ii];
  const int T = d.T;
  const double* prm = g.prm + d.oP;
  const ParamOffsets po = param_offsets(NX, NU, d.n_obs);
  const double* xh = g.xhat + d.oX;
  double* uh = g.uhat + d.oU;
  const double* du = g.du + d.oU;
  const double* dx = g.dx + d.oX;
  double* x1 = g.dx2 + d.oX;    // QP scratch is free after the solve
  double* u1 = g.du2 + d.oU;
  const double* Q = prm + po.Q;
  const double* Ru = prm + po.Ru;
  const double* xg = prm + po.xg;
  __shared__ double red[3 * 16];
  if (threadIdx.x == 0) {
    double x[NX], f[NX];
    for (int i = 0; i < NX; ++i) x[i] = prm[po.x0 + i];
    for (int i = 0; i < NX; ++i) x1[i] = x[i];
    for (int k = 0; k < T; ++k) {
      for (int u = 0; u < NU; ++u) u1[k * NU + u] = uh[k * NU + u] + du[k * NU + u];
      xdot_dev<NX, NU>(d.dyn, prm, po, d.mass, x, u1 + k * NU, f);
      for (int i = 0; i < NX; ++i) x[i] += d.dt * f[i];
      for (int i = 0; i < NX; ++i) x1[(k + 1) * NX + i] = x[i];
    }
  }
  __syncthreads();
  // costs: J(u_hat), Q_u(du), J(u_hat + du)
  double c0 = 0.0, cp = 0.0, c1 = 0.0;
  for (int k = threadIdx.x; k < T; k += blockDim.x) {
    for (int a = 0; a < NU; ++a)
      for (int b = 0; b < NU; ++b) {
        const double r = Ru[a * NU + b];
        c0 += uh[k * NU + a] * r * uh[k * NU + b];
        cp += (uh[k * NU + a] + du[k * NU + a]) * r * (uh[k * NU + b] + du[k * NU + b]);
        c1 += u1[k * NU + a] * r * u1[k * NU + b];
      }
    const int t = k + 1;
    for (int a = 0; a < NX; ++a)
      for (int b = 0; b < NX; ++b) {
        const double q = Q[a * NX + b];
        c0 += (xh[t * NX + a] - xg[a]) * q * (xh[t * NX + b] - xg[b]);
        cp += (xh[t * NX + a] + dx[t * NX + a] - xg[a]) * q * (xh[t * NX + b] + dx[t * NX + b] - xg[b]);
        c1 += (x1[t * NX + a] - xg[a]) * q * (x1[t * NX + b] - xg[b]);
      }
  }
  // penalties
  const double* carr = g.carr;
  const int64_t nc = g.ncones;
  for (int j = threadIdx.x; j < d.ng; j += blockDim.x) {
    const int32_t* m = g.cmeta + (d.cone0 + j) * CM_N;
    const double g0 = carr[(int64_t)CA_G0 * nc + d.cone0 + j];
    const double n = carr[(int64_t)CA_N * nc + d.cone0 + j];
    double lin, gnew;
    if (m[CM_KIND] == 1) {
      const int k = m[CM_TIME], i = m[CM_CIDX], s = m[CM_CSIGN];
      const double bound = (s > 0) ? prm[po.uhi + i] : prm[po.ulo + i];
      lin = s * du[k * NU + i];
      gnew = s * u1[k * NU + i] - s * bound;
    } else {
      const double* w = g.w + d.oW + (int64_t)j * NX;
      const int t = m[CM_TIME];
      lin = 0.0;
      for (int a = 0; a < NX; ++a) lin += w[a] * dx[t * NX + a];
      double wtmp[NX];
      gnew = state_cons_eval<NX, NU>(g, d, j, m, x1 + t * NX, wtmp);
    }
    c0 += w_p * fmax(0.0, g0 + n);
    cp += w_p * fmax(0.0, g0 + lin + n);
    c1 += w_p * fmax(0.0, gnew + n);
  }
  c0 = wave_sum(c0);
  cp = wave_sum(cp);
  c1 = wave_sum(c1);
  if (lane_id() == 0) {
    red[wave_id() * 3 + 0] = c0;
    red[wave_id() * 3 + 1] = cp;
    red[wave_id() * 3 + 2] = c1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double cur = 0.0, pred = 0.0, act = 0.0;
    for (int w = 0; w < (int)(blockDim.x / NRTO_WAVE); ++w) {
      cur += red[w * 3];
      pred += red[w * 3 + 1];
      act += red[w * 3 + 2];
    }
    const double dpred = cur - pred;
    const double ratio = dpred > 0.0 ? (cur - act) / dpred : -1e300;
    const bool acc = g.rep[ii].status == NRTO_OK && dpred > 0.0 && ratio >= 0.1;
    double r = d.r_trust;
    if (acc) {
      if (ratio >= 0.75) r = fmin(1.5 * r, 1e3);
    } else {
      r = fmax(0.8 * r, 1e-3);
    }
    d.r_trust = r;
    out[ii * 5 + 0] = acc ? 1.0 : 0.0;
    out[ii * 5 + 1] = cur;
    out[ii * 5 + 2] = act;
    out[ii * 5 + 3] = pred;
    out[ii * 5 + 4] = r;
    red[47] = acc ? 1.0 : 0.0;
  }
  __syncthreads();
  if (red[47] != 0.0)
    for (int i = threadIdx.x; i < T * NU; i += blockDim.x) uh[i] = u1[i];
}

__global__ void scp_eval_kernel(DevPtrs g, double w_p, double* out) {
  const int ii = blockIdx.x;
  const int nx = g.inst[ii].nx;
  if (nx == 3) scp_eval<3, 2>(g, ii, w_p, out);
  else if (nx == 12) scp_eval<12, 4>(g, ii, w_p, out);
  else scp_eval<14, 7>(g, ii, w_p, out);
}

hipError_t launch_scp_eval(const DevPtrs& g, int n_inst, double w_p, double* out, hipStream_t s) {
  hipLaunchKernelGGL(scp_eval_kernel, dim3(n_inst), dim3(256), 0, s, g, w_p, out);
  return hipGetLastError();
}

hipError_t launch_linearize(const DevPtrs& g, int n_inst, int max_ng, hipStream_t s) {
  hipLaunchKernelGGL(rollout_kernel, dim3(n_inst), dim3(128), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int bx = (max_ng + 127) / 128;
  hipLaunchKernelGGL(cone_data_kernel, dim3(bx > 0 ? bx : 1, n_inst), dim3(128), 0, s, g, n_inst);
  return hipGetLastError();
}

}  // namespace nrto
