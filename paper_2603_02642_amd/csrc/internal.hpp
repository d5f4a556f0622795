// Internal layout shared by the host context code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nrto.h"

namespace nrto {

nrto_status set_global_error(nrto_status s, const std::string& msg);

constexpr int MAX_NX = 14;
constexpr int MAX_NU = 7;
constexpr int MAX_T = 128;

// Per-instance descriptor, resident in device memory.  Offsets are element
// offsets into the concatenated arrays of the context.
struct InstDev {
  int32_t dyn, nx, nu, T;
  int32_t ng, nstate, nent, nblk;
  int32_t ntask, n_obs;
  int32_t nlong;   // wave tasks of one long cone, listed first; the packed tasks follow
  int32_t pad1;
  int64_t cone0;   // first cone (global cone index)
  int64_t ent0;    // first cone entry
  int64_t bv0;     // first element of the block vectors (nu per block)
  int64_t task0;   // first wave task
  int64_t lb0;     // first row of the packed tasks' lane table (64 LaneBlocks a row)
  int64_t oA;      // A: T*nx*nx
  int64_t oB;      // B: T*nx*nu
  int64_t oX;      // xhat: (T+1)*nx  (also dx)
  int64_t oU;      // uhat: T*nu      (also du)
  int64_t oK;      // gains: T*nu*nx  (K, K~, Riccati gains, KKT scratch)
  int64_t oW;      // constraint gradients: ng*nx
  int64_t oP;      // parameters: Q nx*nx, Ru nu*nu, RK2 nu*nu, xg nx, x0 nx, u_lo nu, u_hi nu,
                   //             x_lo nx, x_hi nx, inertia 3, links 7, obstacles n_obs*4
  int64_t oTL;     // time lists: state cones by t (T+2), control cones by k (T+1)
  int64_t oG;      // block Cholesky factors: T*nu*nu
  double radius, r_trust, dt, mass;
};

// Offsets inside the parameter block of one instance.
struct ParamOffsets {
  int Q, Ru, RK2, xg, x0, ulo, uhi, xlo, xhi, inertia, links, obs, size;
};
__host__ __device__ inline ParamOffsets param_offsets(int nx, int nu, int n_obs) {
  ParamOffsets p;
  p.Q = 0;
  p.Ru = p.Q + nx * nx;
  p.RK2 = p.Ru + nu * nu;
  p.xg = p.RK2 + nu * nu;
  p.x0 = p.xg + nx;
  p.ulo = p.x0 + nx;
  p.uhi = p.ulo + nu;
  p.xlo = p.uhi + nu;
  p.xhi = p.xlo + nx;
  p.inertia = p.xhi + nx;
  p.links = p.inertia + 3;
  p.obs = p.links + 7;
  p.size = p.obs + 4 * n_obs;
  return p;
}

// Cone metadata (per cone, int32 x 8): entry offset within the instance, first
// block time, number of blocks, block offset within the instance, kind
// (0 state / 1 control), time (t_j or k_j), control index, control sign.
enum { CM_EOFF = 0, CM_K0, CM_NBLK, CM_BOFF, CM_KIND, CM_TIME, CM_CIDX, CM_CSIGN, CM_N };

// Per-cone float64 arrays in one block of n_cone_arrays * ncones values.
enum {
  CA_G0 = 0,  // g_j at the nominal point
  CA_P,       // p
  CA_PT,      // p~ (last chi)
  CA_PTT,     // DR: p~~ (DR state);  FullADMM: unused
  CA_LAM,     // DR: lambda; FullADMM: lambda_p (scaled)
  CA_PI,      // constraint multiplier pi
  CA_BETA,    // g0 + c (input of the (du, p) block)
  CA_ACT,     // active flag of the (du, p) block (0/1 as double)
  CA_N,       // KKT: ||eta_j||
  CA_ZZ,      // KKT: ||zeta_j||^2
  CA_ZE,      // KKT: zeta_j . eta_j
  CA_E,       // constraint value e_j = g0 + b_j' du
  CA_LA,      // line-search scratch: a_j at the current iterate
  CA_LE,      // line-search scratch: change of a_j along the Newton direction
  CA_PTP,     // p~ of the previous ADMM iteration (dual residual r_d)
  CA_NUM
};

// A wave task: a contiguous run of cones processed by one wavefront.  Either
// one cone longer than 64 entries, or several cones with at most 64 entries
// together (then `mask` marks the cone starts).
struct WaveTask {
  int32_t cone;    // first cone (local index)
  int32_t ncone;
  int32_t ebeg;    // first entry (local index)
  int32_t len;     // entries
  int32_t k0;      // single-cone task: the cone's first block and first block
  int32_t boff;    // vector (its metadata, so that one load describes the task)
  int32_t pad0, pad1;
};

// Block of the entry a lane of a packed wave task holds: block time k and block
// vector index b (local to the instance); k = -1 for a cone's t slot, a block
// without gain (k = T) and the lanes past the task.  Row r of the table serves
// packed task nlong + r of the instance.
struct LaneBlock {
  int32_t k, b;
};

enum { ISCR_PSI = 0, ISCR_KKT, ISCR_RP, ISCR_RD, ISCR_MUHINT, ISCR_N = 8 };

struct SolveOpts {
  int32_t method, precision, max_admm, max_inner, check_every, warm, cold_init, rho_adapt;
  double rho, alpha, sigma_chi, sigma_s, eps_dr_abs, eps_dr_rel, eps_kkt;
  double rho_mu, rho_tau, rho_min, rho_max;
  int32_t sigma_adapt, sigma_every;
  double sigma_thr, sigma_min, sigma_max;
  int32_t infeas_window;
  int32_t cont;   // continuation launch of a solve run in chunks of ADMM iterations (admm_chunk)
};

// Device pointers the kernels use.
struct DevPtrs {
  InstDev* inst;
  int32_t* cmeta;      // ncones * CM_N
  double* carr;        // CA_NUM * ncones
  double* w;           // gradients
  double* bhat64;      // entries
  float* bhat32;
  double* bvec64;      // blocks * nu
  float* bvec32;
  void* st;            // entries, 8 bytes each (DR s~ / FullADMM lambda_nu)
  void* nu;            // entries, 8 bytes each (FullADMM nu)
  double* A;
  double* B;
  double* xhat;
  double* uhat;
  double* dx;          // QP iterate states ((T+1)*nx)
  double* du;          // QP iterate controls
  double* dx2;         // QP candidate states
  double* du2;         // QP candidate controls
  double* K;           // gains (double)
  double* Kt;          // DR K~
  double* kscr;        // KKT accumulation of sum_j A_hat_j' zeta_j (double)
  double* prm;
  int32_t* tl;
  double* gch;
  WaveTask* tasks;
  uint64_t* tmask;
  LaneBlock* lblock;   // packed tasks' lane table
  double* mu;          // per instance trust-region multiplier
  double* iscr;        // per instance scratch, ISCR_N doubles
  int32_t* flags;      // per instance: [0] lambda_nu update pending
  nrto_solve_report* rep;
  int64_t ncones;
};

}  // namespace nrto
