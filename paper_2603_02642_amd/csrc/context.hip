// Host side of the C ABI: context creation, compact cone layout, wave task
// schedule, host <-> device transfers and solver launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace nrto {

size_t solver_smem_bytes(int T, int nx, int nu, int precision, int threads);
hipError_t launch_solver(const DevPtrs& g, const SolveOpts& o, int nx, const int32_t* order, int n, int threads,
                         size_t smem, hipStream_t s);
hipError_t set_solver_smem_limit(size_t bytes);
hipError_t launch_warm(const DevPtrs& g, const SolveOpts& o, int nx, const int32_t* order, int n, int threads,
                       size_t smem, const float* pred, int64_t ld, int test, int32_t* acc, double* res, hipStream_t s);
hipError_t launch_linearize(const DevPtrs& g, int n_inst, int max_ng, hipStream_t s);
hipError_t launch_scp_eval(const DevPtrs& g, int n_inst, double w_p, double* out, hipStream_t s);

static thread_local std::string g_err;

nrto_status set_global_error(nrto_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace nrto

using namespace nrto;

struct HostInst {
  InstDev d;
  std::vector<int32_t> cmeta;
  std::vector<WaveTask> tasks;
  std::vector<uint64_t> tmask;
  std::vector<LaneBlock> lblock;   // 64 per packed task
  std::vector<int32_t> tl;
  std::vector<double> prm;
  std::vector<double> uinit;
};

struct nrto_ctx_s {
  hipStream_t stream = nullptr;
  nrto_options opt{};
  int n = 0;
  std::vector<HostInst> hi;
  DevPtrs g{};
  std::vector<void*> allocs;
  int64_t ncones = 0, nent = 0, nbv = 0, nA = 0, nB = 0, nX = 0, nU = 0, nK = 0, nW = 0, nP = 0, nTL = 0,
          nG = 0, ntask = 0, nlb = 0;
  int32_t* order = nullptr;
  std::vector<int32_t> horder;
  int group_nx[3] = {3, 12, 14};
  int group_off[4] = {0, 0, 0, 0};   // instances of model g are order[group_off[g] .. group_off[g+1])
  int threads = 256;
  size_t smem = 0;
  std::string err;
  std::vector<double> rtrust;  // per-instance trust radius (host copy)
  double* scp_out = nullptr;   // 5 per instance: merit-test results of nrto_scp_step
  double us_per_tick = 0.0;    // device wall clock period in microseconds
  hipGraphExec_t step_exec = nullptr;  // captured linearise + solve (nrto_capture_step)
  hipStream_t aux[2] = {nullptr, nullptr};  // the second and third model groups' solve launches
  hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
  int32_t* ws_acc = nullptr;   // nrto_warm_start: accepted flag per instance
  double* ws_res = nullptr;    // nrto_warm_start: (warm, cold) residual per instance
};

// Scale the wall-clock tick counts of device-written reports to microseconds.
static void reports_to_us(const nrto_ctx c, nrto_solve_report* r, int n) {
  for (int i = 0; i < n; ++i) {
    r[i].t_dr_us *= c->us_per_tick;
    r[i].t_qp_us *= c->us_per_tick;
    r[i].t_kkt_us *= c->us_per_tick;
    r[i].t_total_us *= c->us_per_tick;
  }
}

static nrto_status ctx_err(nrto_ctx c, nrto_status s, const std::string& m) {
  if (c) c->err = m;
  g_err = m;
  return s;
}

#define HIPCHK(ctx, expr)                                                            \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) return ctx_err(ctx, NRTO_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

template <typename T>
static nrto_status dalloc(nrto_ctx c, T** p, int64_t n) {
  size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
  void* q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess)
    return ctx_err(c, NRTO_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  c->allocs.push_back(q);
  if (hipMemsetAsync(q, 0, bytes, c->stream) != hipSuccess) return ctx_err(c, NRTO_ERR_HIP, "hipMemsetAsync failed");
  *p = (T*)q;
  return NRTO_OK;
}

extern "C" void nrto_default_options(nrto_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = NRTO_DR;
  o->precision = NRTO_FP64;
  o->max_admm = 40;
  o->max_inner = 100;
  o->check_every = 1;
  o->block_threads = 0;
  o->rho = 40.0;
  o->alpha = 1.0;
  o->sigma_chi = 1.0;
  o->sigma_s = 1.0;
  o->eps_dr_abs = 1e-4;
  o->eps_dr_rel = 1e-4;
  o->eps_kkt = 1e-4;
  o->r_trust = 2.0;
  o->cold_init = 0;
  o->rho_adapt = 0;
  o->rho_mu = 10.0;
  o->rho_tau = 2.0;
  o->rho_min = 1.0;
  o->rho_max = 200.0;
  o->sigma_adapt = 0;
  o->sigma_every = 10;
  o->sigma_thr = 5.0;
  o->sigma_min = 1e-4;
  o->sigma_max = 1e6;
}

extern "C" const char* nrto_last_error(nrto_ctx c) { return c ? c->err.c_str() : g_err.c_str(); }

static bool finite_or_inf(double v) { return !std::isnan(v); }

// Build the structural layout of one problem.
static nrto_status build_instance(nrto_ctx c, const nrto_problem& p, HostInst& h) {
  const int nx = p.nx, nu = p.nu, T = p.T;
  bool ok = (p.dyn == NRTO_DYN_UNICYCLE && nx == 3 && nu == 2) || (p.dyn == NRTO_DYN_QUADROTOR && nx == 12 && nu == 4) ||
            (p.dyn == NRTO_DYN_ARM && nx == 14 && nu == 7);
  if (!ok) return ctx_err(c, NRTO_ERR_ARG, "dyn/nx/nu must be unicycle (3,2), quadrotor (12,4) or arm (14,7)");
  if (T < 1 || T > MAX_T) return ctx_err(c, NRTO_ERR_ARG, "T must be in [1, 128]");
  if (!p.x0 || !p.xg || !p.Q || !p.Ru || !p.RK || !p.u_init) return ctx_err(c, NRTO_ERR_ARG, "null problem array");
  if (p.n_obs < 0 || (p.n_obs > 0 && !p.obs)) return ctx_err(c, NRTO_ERR_ARG, "bad obstacles");
  if (!(p.radius >= 0.0) || !(p.dt > 0.0)) return ctx_err(c, NRTO_ERR_ARG, "radius >= 0 and dt > 0 required");
  if (p.dyn == NRTO_DYN_QUADROTOR && (!p.inertia || !(p.mass > 0.0))) return ctx_err(c, NRTO_ERR_ARG, "quadrotor needs mass and inertia");
  if (p.dyn == NRTO_DYN_ARM && !p.links) return ctx_err(c, NRTO_ERR_ARG, "arm needs links");
  const int npts = (p.dyn == NRTO_DYN_ARM) ? 7 : 1;
  // constraints per time
  std::vector<int32_t> cm;
  int ent = 0, blk = 0, nstate = 0;
  std::vector<int32_t> tls(T + 2, 0), tlc(T + 1, 0);
  auto add = [&](int kind, int time, int k0, int nblk, int cidx, int csign) {
    int32_t m[CM_N];
    m[CM_EOFF] = ent;
    m[CM_K0] = k0;
    m[CM_NBLK] = nblk;
    m[CM_BOFF] = blk;
    m[CM_KIND] = kind;
    m[CM_TIME] = time;
    m[CM_CIDX] = cidx;
    m[CM_CSIGN] = csign;
    cm.insert(cm.end(), m, m + CM_N);
    ent += 1 + nblk * nx;
    blk += nblk;
  };
  for (int t = 1; t <= T; ++t) {
    tls[t] = (int)(cm.size() / CM_N);
    for (int o = 0; o < p.n_obs; ++o)
      for (int q = 0; q < npts; ++q) add(0, t, 0, t + 1, -1, 0);
    if (p.x_hi && p.x_lo)
      for (int i = 0; i < nx; ++i) {
        if (std::isfinite(p.x_hi[i])) add(0, t, 0, t + 1, i, 1);
        if (std::isfinite(p.x_lo[i])) add(0, t, 0, t + 1, i, -1);
      }
  }
  nstate = (int)(cm.size() / CM_N);
  tls[0] = 0;
  tls[T + 1] = nstate;
  for (int k = 0; k < T; ++k) {
    tlc[k] = (int)(cm.size() / CM_N);
    for (int i = 0; i < nu; ++i) {
      if (p.u_hi && std::isfinite(p.u_hi[i])) add(1, k, k, 1, i, 1);
      if (p.u_lo && std::isfinite(p.u_lo[i])) add(1, k, k, 1, i, -1);
    }
  }
  const int ng = (int)(cm.size() / CM_N);
  tlc[T] = ng;
  for (int i = 0; i < ng; ++i)
    if (c->opt.method == NRTO_FULLADMM && 1 + cm[i * CM_N + CM_NBLK] * nx > 64 * 16)
      return ctx_err(c, NRTO_ERR_ARG, "FullADMM: cone longer than 1024 entries (reduce T)");
  // wave tasks: long cones alone, short consecutive cones packed up to 64 entries
  std::vector<WaveTask> longt, shortt;
  std::vector<uint64_t> shortm;
  {
    int j = 0;
    while (j < ng) {
      int len = 1 + cm[j * CM_N + CM_NBLK] * nx;
      if (len > 64) {
        longt.push_back({j, 1, cm[j * CM_N + CM_EOFF], len, cm[j * CM_N + CM_K0], cm[j * CM_N + CM_BOFF], 0, 0});
        ++j;
        continue;
      }
      WaveTask tk{j, 0, cm[j * CM_N + CM_EOFF], 0, 0, 0, 0, 0};
      uint64_t mask = 0;
      while (j < ng) {
        int l2 = 1 + cm[j * CM_N + CM_NBLK] * nx;
        if (l2 > 64 || tk.len + l2 > 64) break;
        mask |= (1ull << tk.len);
        tk.len += l2;
        tk.ncone += 1;
        ++j;
      }
      shortt.push_back(tk);
      shortm.push_back(mask);
    }
  }
  std::sort(longt.begin(), longt.end(), [](const WaveTask& a, const WaveTask& b) { return a.len > b.len; });
  h.tasks = longt;
  h.tmask.assign(longt.size(), 0ull);
  h.tasks.insert(h.tasks.end(), shortt.begin(), shortt.end());
  h.tmask.insert(h.tmask.end(), shortm.begin(), shortm.end());
  // lane table of the packed tasks: the block time and block vector of each lane's entry
  h.lblock.assign(shortt.size() * 64, LaneBlock{-1, -1});
  for (size_t s = 0; s < shortt.size(); ++s) {
    const WaveTask& tk = shortt[s];
    int c = tk.cone;
    for (int l = 0; l < tk.len; ++l) {
      const int e = tk.ebeg + l;
      while (c + 1 < tk.cone + tk.ncone && cm[(c + 1) * CM_N + CM_EOFF] <= e) ++c;
      const int le = e - cm[c * CM_N + CM_EOFF];
      if (le == 0) continue;
      const int blk = (le - 1) / nx;
      const int k = cm[c * CM_N + CM_K0] + blk;
      if (k < T) h.lblock[s * 64 + l] = LaneBlock{k, cm[c * CM_N + CM_BOFF] + blk};
    }
  }
  h.cmeta = cm;
  h.tl = tls;
  h.tl.insert(h.tl.end(), tlc.begin(), tlc.end());
  // parameters
  ParamOffsets po = param_offsets(nx, nu, p.n_obs);
  h.prm.assign(po.size, 0.0);
  for (int i = 0; i < nx * nx; ++i) h.prm[po.Q + i] = p.Q[i];
  for (int i = 0; i < nu * nu; ++i) h.prm[po.Ru + i] = p.Ru[i];
  for (int u = 0; u < nu; ++u)
    for (int w = 0; w < nu; ++w) {
      double s = 0.0;
      for (int l = 0; l < nu; ++l) s += p.RK[l * nu + u] * p.RK[l * nu + w];
      h.prm[po.RK2 + u * nu + w] = s;
    }
  for (int i = 0; i < nx; ++i) {
    h.prm[po.xg + i] = p.xg[i];
    h.prm[po.x0 + i] = p.x0[i];
    h.prm[po.xlo + i] = (p.x_lo ? p.x_lo[i] : -INFINITY);
    h.prm[po.xhi + i] = (p.x_hi ? p.x_hi[i] : INFINITY);
  }
  for (int i = 0; i < nu; ++i) {
    h.prm[po.ulo + i] = (p.u_lo ? p.u_lo[i] : -INFINITY);
    h.prm[po.uhi + i] = (p.u_hi ? p.u_hi[i] : INFINITY);
  }
  if (p.inertia)
    for (int i = 0; i < 3; ++i) h.prm[po.inertia + i] = p.inertia[i];
  if (p.links)
    for (int i = 0; i < 7; ++i) h.prm[po.links + i] = p.links[i];
  const int od = (p.dyn == NRTO_DYN_UNICYCLE) ? 2 : 3;
  for (int o = 0; o < p.n_obs; ++o) {
    for (int i = 0; i < od; ++i) h.prm[po.obs + 4 * o + i] = p.obs[o * (od + 1) + i];
    h.prm[po.obs + 4 * o + 3] = p.obs[o * (od + 1) + od];
  }
  h.uinit.assign(p.u_init, p.u_init + T * nu);
  InstDev& d = h.d;
  std::memset(&d, 0, sizeof(d));
  d.dyn = p.dyn;
  d.nx = nx;
  d.nu = nu;
  d.T = T;
  d.ng = ng;
  d.nstate = nstate;
  d.nent = ent;
  d.nblk = blk;
  d.ntask = (int)h.tasks.size();
  d.nlong = (int)longt.size();
  d.n_obs = p.n_obs;
  d.radius = p.radius;
  d.dt = p.dt;
  d.mass = p.mass;
  return NRTO_OK;
}

static void fill_opts(const nrto_ctx c, SolveOpts& o, int warm) {
  o.method = c->opt.method;
  o.precision = c->opt.precision;
  o.max_admm = c->opt.max_admm;
  o.max_inner = c->opt.max_inner;
  o.check_every = std::max(1, c->opt.check_every);
  o.warm = warm;
  o.rho = c->opt.rho;
  o.alpha = c->opt.alpha;
  o.sigma_chi = c->opt.sigma_chi;
  o.sigma_s = c->opt.sigma_s;
  o.eps_dr_abs = c->opt.eps_dr_abs;
  o.eps_dr_rel = c->opt.eps_dr_rel;
  o.eps_kkt = c->opt.eps_kkt;
  o.cold_init = c->opt.cold_init;
  o.rho_adapt = c->opt.rho_adapt;
  o.rho_mu = c->opt.rho_mu;
  o.rho_tau = c->opt.rho_tau;
  o.rho_min = c->opt.rho_min;
  o.rho_max = c->opt.rho_max;
  o.sigma_adapt = c->opt.sigma_adapt;
  o.sigma_every = c->opt.sigma_every;
  o.sigma_thr = c->opt.sigma_thr;
  o.sigma_min = c->opt.sigma_min;
  o.sigma_max = c->opt.sigma_max;
  o.infeas_window = c->opt.infeas_window;
  o.cont = 0;
}

static nrto_status check_options(nrto_ctx c, const nrto_options* o) {
  if (!o) return ctx_err(c, NRTO_ERR_ARG, "null options");
  if (o->method != NRTO_DR && o->method != NRTO_FULLADMM) return ctx_err(c, NRTO_ERR_ARG, "bad method");
  if (o->precision != NRTO_FP64 && o->precision != NRTO_FP32) return ctx_err(c, NRTO_ERR_ARG, "bad precision");
  if (o->max_admm < 1 || o->max_inner < 1) return ctx_err(c, NRTO_ERR_ARG, "iteration limits must be >= 1");
  if (!(o->rho > 0) || !(o->alpha > 0 && o->alpha < 2) || !(o->sigma_chi > 0) || !(o->sigma_s > 0))
    return ctx_err(c, NRTO_ERR_ARG, "rho, sigma > 0 and alpha in (0, 2) required");
  if (!(o->r_trust > 0)) return ctx_err(c, NRTO_ERR_ARG, "r_trust > 0 required");
  if (o->block_threads != 0 && (o->block_threads < 64 || o->block_threads > 1024 || o->block_threads % 64))
    return ctx_err(c, NRTO_ERR_ARG, "block_threads must be 0 or a multiple of 64 in [64, 1024]");
  if (o->cold_init != 0 && o->cold_init != 1) return ctx_err(c, NRTO_ERR_ARG, "cold_init must be 0 or 1");
  if (o->infeas_window < 0) return ctx_err(c, NRTO_ERR_ARG, "infeas_window must be >= 0");
  if (o->admm_chunk < 0) return ctx_err(c, NRTO_ERR_ARG, "admm_chunk must be >= 0");
  if (o->rho_adapt != 0 && o->rho_adapt != 1) return ctx_err(c, NRTO_ERR_ARG, "rho_adapt must be 0 or 1");
  if (o->rho_adapt &&
      !(o->rho_mu > 1 && o->rho_tau > 1 && o->rho_min > 0 && o->rho_min <= o->rho && o->rho <= o->rho_max))
    return ctx_err(c, NRTO_ERR_ARG, "rho_adapt needs rho_mu > 1, rho_tau > 1, 0 < rho_min <= rho <= rho_max");
  if (o->sigma_adapt != 0 && o->sigma_adapt != 1) return ctx_err(c, NRTO_ERR_ARG, "sigma_adapt must be 0 or 1");
  if (o->sigma_adapt && !(o->sigma_every >= 1 && o->sigma_thr > 1 && o->sigma_min > 0 &&
                          o->sigma_min <= o->sigma_s && o->sigma_s <= o->sigma_max))
    return ctx_err(c, NRTO_ERR_ARG,
                   "sigma_adapt needs sigma_every >= 1, sigma_thr > 1, 0 < sigma_min <= sigma_s <= sigma_max");
  return NRTO_OK;
}

static nrto_status configure_launch(nrto_ctx c) {
  int th = c->opt.block_threads;
  if (th == 0) th = (c->n <= 64) ? 512 : 256;
  if (th > 512) return ctx_err(c, NRTO_ERR_ARG, "block_threads above 512 exceeds the solver kernels' launch bound of 512 work-items");
  size_t smem = 0;
  for (auto& h : c->hi) smem = std::max(smem, solver_smem_bytes(h.d.T, h.d.nx, h.d.nu, c->opt.precision, th));
  if (smem > 160 * 1024) return ctx_err(c, NRTO_ERR_ARG, "per-instance LDS need exceeds 160 KB (reduce T or use FP32)");
  c->threads = th;
  c->smem = smem;
  HIPCHK(c, set_solver_smem_limit(smem));
  return NRTO_OK;
}

extern "C" nrto_status nrto_set_options(nrto_ctx c, const nrto_options* o) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  nrto_status s = check_options(c, o);
  if (s != NRTO_OK) return s;
  if (c->step_exec) {
    HIPCHK(c, hipGraphExecDestroy(c->step_exec));   // its kernels carry the old options
    c->step_exec = nullptr;
  }
  const nrto_options prev = c->opt;
  c->opt = *o;
  if (o->block_threads != prev.block_threads || o->precision != prev.precision) {
    s = configure_launch(c);       // workgroup size and LDS of the launches
    if (s != NRTO_OK) {
      c->opt = prev;
      (void)configure_launch(c);
      return s;
    }
  }
  std::vector<InstDev> d(c->n);
  for (int i = 0; i < c->n; ++i) {
    c->hi[i].d.r_trust = o->r_trust;
    d[i] = c->hi[i].d;
  }
  HIPCHK(c, hipMemcpyAsync(c->g.inst, d.data(), sizeof(InstDev) * c->n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return configure_launch(c);
}

extern "C" nrto_status nrto_setup(const nrto_problem* probs, int32_t n, const nrto_options* opt, void* stream,
                                  nrto_ctx* out) {
  if (!out) return set_global_error(NRTO_ERR_ARG, "null output");
  *out = nullptr;
  if (!probs || n < 1) return set_global_error(NRTO_ERR_ARG, "need at least one problem");
  nrto_ctx c = new (std::nothrow) nrto_ctx_s();
  if (!c) return set_global_error(NRTO_ERR_ALLOC, "out of host memory");
  c->stream = (hipStream_t)stream;
  c->n = n;
  nrto_options o;
  if (opt) o = *opt; else nrto_default_options(&o);
  nrto_status s = check_options(c, &o);
  if (s != NRTO_OK) { g_err = c->err; delete c; return s; }
  c->opt = o;
  c->hi.resize(n);
  for (int i = 0; i < n; ++i) {
    s = build_instance(c, probs[i], c->hi[i]);
    if (s != NRTO_OK) { g_err = "instance " + std::to_string(i) + ": " + c->err; delete c; return s; }
    c->hi[i].d.r_trust = o.r_trust;
  }
  // offsets
  for (auto& h : c->hi) {
    InstDev& d = h.d;
    d.cone0 = c->ncones; c->ncones += d.ng;
    d.ent0 = c->nent; c->nent += d.nent;
    d.bv0 = c->nbv; c->nbv += (int64_t)d.nblk * d.nu;
    d.task0 = c->ntask; c->ntask += d.ntask;
    d.lb0 = c->nlb; c->nlb += (int64_t)(d.ntask - d.nlong);
    d.oA = c->nA; c->nA += (int64_t)d.T * d.nx * d.nx;
    d.oB = c->nB; c->nB += (int64_t)d.T * d.nx * d.nu;
    d.oX = c->nX; c->nX += (int64_t)(d.T + 1) * d.nx;
    d.oU = c->nU; c->nU += (int64_t)d.T * d.nu;
    d.oK = c->nK; c->nK += (int64_t)d.T * d.nu * d.nx;
    d.oW = c->nW; c->nW += (int64_t)d.ng * d.nx;
    d.oP = c->nP; c->nP += (int64_t)h.prm.size();
    d.oTL = c->nTL; c->nTL += (int64_t)h.tl.size();
    d.oG = c->nG; c->nG += (int64_t)d.T * d.nu * d.nu;
  }
  DevPtrs& g = c->g;
  g.ncones = c->ncones;
#define ALLOC(ptr, n)                                       \
  do {                                                      \
    nrto_status _s = dalloc(c, &(ptr), (n));                \
    if (_s != NRTO_OK) { g_err = c->err; nrto_destroy(c); return _s; } \
  } while (0)
  ALLOC(g.inst, n);
  ALLOC(g.cmeta, c->ncones * CM_N);
  ALLOC(g.carr, c->ncones * CA_NUM);
  ALLOC(g.w, c->nW);
  ALLOC(g.bhat64, c->nent);
  ALLOC(g.bhat32, c->nent);
  ALLOC(g.bvec64, c->nbv);
  ALLOC(g.bvec32, c->nbv);
  double* st = nullptr;
  double* nu = nullptr;
  ALLOC(st, c->nent);
  ALLOC(nu, c->nent);
  g.st = st;
  g.nu = nu;
  ALLOC(g.A, c->nA);
  ALLOC(g.B, c->nB);
  ALLOC(g.xhat, c->nX);
  ALLOC(g.uhat, c->nU);
  ALLOC(g.dx, c->nX);
  ALLOC(g.du, c->nU);
  ALLOC(g.dx2, c->nX);
  ALLOC(g.du2, c->nU);
  ALLOC(g.K, c->nK);
  ALLOC(g.Kt, c->nK);
  ALLOC(g.kscr, c->nK);
  ALLOC(g.prm, c->nP);
  ALLOC(g.tl, c->nTL);
  ALLOC(g.gch, c->nG);
  ALLOC(g.tasks, c->ntask);
  ALLOC(g.tmask, c->ntask);
  ALLOC(g.lblock, c->nlb * 64);
  ALLOC(g.mu, n);
  ALLOC(g.iscr, (int64_t)n * ISCR_N);
  ALLOC(g.flags, (int64_t)n * 4);
  ALLOC(g.rep, n);
  ALLOC(c->scp_out, 5 * (int64_t)n);
  ALLOC(c->ws_acc, n);
  ALLOC(c->ws_res, 2 * (int64_t)n);
  ALLOC(c->order, n);
#undef ALLOC
  // uploads
  std::vector<InstDev> d(n);
  std::vector<int32_t> cm;
  std::vector<WaveTask> tk;
  std::vector<uint64_t> tm;
  std::vector<LaneBlock> lb;
  std::vector<int32_t> tl;
  std::vector<double> prm, u;
  for (int i = 0; i < n; ++i) {
    auto& h = c->hi[i];
    d[i] = h.d;
    cm.insert(cm.end(), h.cmeta.begin(), h.cmeta.end());
    tk.insert(tk.end(), h.tasks.begin(), h.tasks.end());
    tm.insert(tm.end(), h.tmask.begin(), h.tmask.end());
    lb.insert(lb.end(), h.lblock.begin(), h.lblock.end());
    tl.insert(tl.end(), h.tl.begin(), h.tl.end());
    prm.insert(prm.end(), h.prm.begin(), h.prm.end());
    u.insert(u.end(), h.uinit.begin(), h.uinit.end());
  }
  // instance order: grouped by model, largest first inside a group (longest processing time first)
  c->horder.resize(n);
  std::iota(c->horder.begin(), c->horder.end(), 0);
  auto grp = [&](int i) { int nx = c->hi[i].d.nx; return nx == 3 ? 0 : (nx == 12 ? 1 : 2); };
  std::stable_sort(c->horder.begin(), c->horder.end(), [&](int a, int b) {
    if (grp(a) != grp(b)) return grp(a) < grp(b);
    return c->hi[a].d.nent > c->hi[b].d.nent;
  });
  for (int gi = 0; gi < 3; ++gi) {
    int cnt = 0;
    for (int i = 0; i < n; ++i) cnt += (grp(i) == gi);
    c->group_off[gi + 1] = c->group_off[gi] + cnt;
  }
  hipStream_t sm = c->stream;
  auto H2D = [&](void* dst, const void* src, size_t bytes) { return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, sm); };
  HIPCHK(c, H2D(g.inst, d.data(), sizeof(InstDev) * n));
  HIPCHK(c, H2D(g.cmeta, cm.data(), sizeof(int32_t) * cm.size()));
  HIPCHK(c, H2D(g.tasks, tk.data(), sizeof(WaveTask) * tk.size()));
  HIPCHK(c, H2D(g.tmask, tm.data(), sizeof(uint64_t) * tm.size()));
  if (!lb.empty()) HIPCHK(c, H2D(g.lblock, lb.data(), sizeof(LaneBlock) * lb.size()));
  HIPCHK(c, H2D(g.tl, tl.data(), sizeof(int32_t) * tl.size()));
  HIPCHK(c, H2D(g.prm, prm.data(), sizeof(double) * prm.size()));
  HIPCHK(c, H2D(g.uhat, u.data(), sizeof(double) * u.size()));
  HIPCHK(c, H2D(c->order, c->horder.data(), sizeof(int32_t) * n));
  HIPCHK(c, hipStreamSynchronize(sm));
  s = configure_launch(c);
  if (s != NRTO_OK) { g_err = c->err; nrto_destroy(c); return s; }
  // side streams (default priority) for the solve launches of the other model groups
  {
    hipError_t e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    for (int j = 0; j < 2 && e == hipSuccess; ++j) {
      e = hipStreamCreateWithFlags(&c->aux[j], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join[j], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      ctx_err(c, NRTO_ERR_HIP, std::string("side streams: ") + hipGetErrorString(e));
      nrto_destroy(c);
      return NRTO_ERR_HIP;
    }
  }
  {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
        khz > 0)
      c->us_per_tick = 1000.0 / (double)khz;
  }
  *out = c;
  return NRTO_OK;
}

extern "C" void nrto_destroy(nrto_ctx c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  for (int j = 0; j < 2; ++j) {
    if (c->aux[j]) (void)hipStreamDestroy(c->aux[j]);
    if (c->ev_join[j]) (void)hipEventDestroy(c->ev_join[j]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
}

extern "C" nrto_status nrto_instance_sizes(nrto_ctx c, int32_t inst, int64_t out[7]) {
  if (!c || !out) return set_global_error(NRTO_ERR_ARG, "null argument");
  if (inst < 0 || inst >= c->n) return ctx_err(c, NRTO_ERR_ARG, "instance out of range");
  const InstDev& d = c->hi[inst].d;
  out[0] = d.ng;
  out[1] = d.nent;
  out[2] = d.nblk;
  out[3] = d.nstate;
  out[4] = d.T;
  out[5] = d.nx;
  out[6] = d.nu;
  return NRTO_OK;
}

template <typename T>
static hipError_t copy_in(T* dst, const T* src, size_t n, hipStream_t s) {
  if (!src || n == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s);
}
template <typename T>
static hipError_t copy_out(T* dst, const T* src, size_t n, hipStream_t s) {
  if (!dst || n == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s);
}

extern "C" nrto_status nrto_upload_socp(nrto_ctx c, int32_t inst, const double* A, const double* B,
                                        const double* xhat, const double* uhat, const double* g0,
                                        const double* w, const double* bhat, const double* bvec) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (inst < 0 || inst >= c->n) return ctx_err(c, NRTO_ERR_ARG, "instance out of range");
  const InstDev& d = c->hi[inst].d;
  hipStream_t s = c->stream;
  HIPCHK(c, copy_in(c->g.A + d.oA, A, (size_t)d.T * d.nx * d.nx, s));
  HIPCHK(c, copy_in(c->g.B + d.oB, B, (size_t)d.T * d.nx * d.nu, s));
  HIPCHK(c, copy_in(c->g.xhat + d.oX, xhat, (size_t)(d.T + 1) * d.nx, s));
  HIPCHK(c, copy_in(c->g.uhat + d.oU, uhat, (size_t)d.T * d.nu, s));
  HIPCHK(c, copy_in(c->g.w + d.oW, w, (size_t)d.ng * d.nx, s));
  if (g0) {
    HIPCHK(c, copy_in(c->g.carr + (int64_t)CA_G0 * c->ncones + d.cone0, g0, (size_t)d.ng, s));
  }
  std::vector<float> f;
  if (bhat) {
    HIPCHK(c, copy_in(c->g.bhat64 + d.ent0, bhat, (size_t)d.nent, s));
    f.assign(bhat, bhat + d.nent);
    HIPCHK(c, copy_in(c->g.bhat32 + d.ent0, f.data(), (size_t)d.nent, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  if (bvec) {
    const size_t nb = (size_t)d.nblk * d.nu;
    HIPCHK(c, copy_in(c->g.bvec64 + d.bv0, bvec, nb, s));
    f.assign(bvec, bvec + nb);
    HIPCHK(c, copy_in(c->g.bvec32 + d.bv0, f.data(), nb, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return NRTO_OK;
}

extern "C" nrto_status nrto_download_socp(nrto_ctx c, int32_t inst, double* A, double* B, double* xhat,
                                          double* uhat, double* g0, double* w, double* bhat, double* bvec) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (inst < 0 || inst >= c->n) return ctx_err(c, NRTO_ERR_ARG, "instance out of range");
  const InstDev& d = c->hi[inst].d;
  hipStream_t s = c->stream;
  HIPCHK(c, copy_out(A, c->g.A + d.oA, (size_t)d.T * d.nx * d.nx, s));
  HIPCHK(c, copy_out(B, c->g.B + d.oB, (size_t)d.T * d.nx * d.nu, s));
  HIPCHK(c, copy_out(xhat, c->g.xhat + d.oX, (size_t)(d.T + 1) * d.nx, s));
  HIPCHK(c, copy_out(uhat, c->g.uhat + d.oU, (size_t)d.T * d.nu, s));
  HIPCHK(c, copy_out(g0, c->g.carr + (int64_t)CA_G0 * c->ncones + d.cone0, (size_t)d.ng, s));
  HIPCHK(c, copy_out(w, c->g.w + d.oW, (size_t)d.ng * d.nx, s));
  HIPCHK(c, copy_out(bhat, c->g.bhat64 + d.ent0, (size_t)d.nent, s));
  HIPCHK(c, copy_out(bvec, c->g.bvec64 + d.bv0, (size_t)d.nblk * d.nu, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return NRTO_OK;
}

// Solve launches of all model groups: the first non-empty group on the context's
// stream, the others on side streams forked from and joined back into it, so
// that the groups' persistent launches overlap (their tails in particular).
static nrto_status launch_solve(nrto_ctx c, int warm, const DevPtrs& g) {
  SolveOpts o;
  fill_opts(c, o, warm);
  int groups[3], ng = 0;
  for (int gi = 0; gi < 3; ++gi)
    if (c->group_off[gi + 1] > c->group_off[gi]) groups[ng++] = gi;
  // chunked solve: launches of at most admm_chunk ADMM iterations; the later
  // ones continue the instances that have not stopped (a fixed number of
  // launches, so a captured step replays them all)
  const int total = c->opt.max_admm;
  const int chunk = (c->opt.admm_chunk > 0 && c->opt.admm_chunk < total) ? c->opt.admm_chunk : total;
  for (int done = 0; done < total; done += chunk) {
    o.max_admm = std::min(chunk, total - done);
    o.cont = done > 0 ? 1 : 0;
    o.warm = done > 0 ? 1 : warm;
    if (ng > 1) HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
    for (int j = 0; j < ng; ++j) {
      const int gi = groups[j];
      hipStream_t s = (j == 0) ? c->stream : c->aux[j - 1];
      if (j > 0) HIPCHK(c, hipStreamWaitEvent(s, c->ev_fork, 0));
      const int cnt = c->group_off[gi + 1] - c->group_off[gi];
      HIPCHK(c, launch_solver(g, o, c->group_nx[gi], c->order + c->group_off[gi], cnt, c->threads, c->smem, s));
      if (j > 0) {
        HIPCHK(c, hipEventRecord(c->ev_join[j - 1], s));
        HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join[j - 1], 0));
      }
    }
  }
  return NRTO_OK;
}

extern "C" nrto_status nrto_solve_socp(nrto_ctx c, int32_t warm, nrto_solve_report* rep) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (c->opt.method == NRTO_FULLADMM)
    return ctx_err(c, NRTO_ERR_STATE,
                   "the FullADMM device path is switched off: its kernel took a GPU memory fault whose cause "
                   "is not yet identified; use NRTO_DR");
  if (c->opt.precision == NRTO_FP32)
    return ctx_err(c, NRTO_ERR_STATE,
                   "the FP32 solver path is switched off: its kernel took a GPU memory fault whose cause is not "
                   "yet identified; use NRTO_FP64");
  nrto_status ls = launch_solve(c, warm ? 1 : 0, c->g);
  if (ls != NRTO_OK) return ls;
  if (rep) {
    HIPCHK(c, copy_out(rep, c->g.rep, (size_t)c->n, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    reports_to_us(c, rep, c->n);
  }
  return NRTO_OK;
}

extern "C" nrto_status nrto_solve_socp_dev(nrto_ctx c, const nrto_socp_dev* sd, nrto_socp_state_dev* st,
                                           int32_t warm, nrto_solve_report* rep) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (!sd || !st) return ctx_err(c, NRTO_ERR_ARG, "null SOCP or state view");
  if (!sd->A || !sd->B || !sd->xhat || !sd->uhat || !sd->g0 || !sd->w || !sd->bhat || !sd->bvec)
    return ctx_err(c, NRTO_ERR_ARG, "null SOCP array");
  if (!st->st || !st->kt || !st->ptt || !st->du || !st->K || !st->p || !st->pt || !st->lam || !st->pi)
    return ctx_err(c, NRTO_ERR_ARG, "null state array");
  if (c->opt.method != NRTO_DR || c->opt.precision != NRTO_FP64)
    return ctx_err(c, NRTO_ERR_STATE, "nrto_solve_socp_dev runs NRTO-DR in FP64");
  DevPtrs g = c->g;
  g.A = const_cast<double*>(sd->A);
  g.B = const_cast<double*>(sd->B);
  g.xhat = const_cast<double*>(sd->xhat);
  g.uhat = const_cast<double*>(sd->uhat);
  g.w = const_cast<double*>(sd->w);
  g.bhat64 = const_cast<double*>(sd->bhat);
  g.bvec64 = const_cast<double*>(sd->bvec);
  g.st = st->st;
  g.Kt = st->kt;
  g.K = st->K;
  g.du = st->du;
  hipStream_t s = c->stream;
  const size_t nc = (size_t)c->ncones;
  auto col = [&](int k) { return c->g.carr + (int64_t)k * c->ncones; };
  auto d2d = [&](double* dst, const double* src) {
    return hipMemcpyAsync(dst, src, nc * sizeof(double), hipMemcpyDeviceToDevice, s);
  };
  HIPCHK(c, d2d(col(CA_G0), sd->g0));
  if (warm) {
    HIPCHK(c, d2d(col(CA_P), st->p));
    HIPCHK(c, d2d(col(CA_PT), st->pt));
    HIPCHK(c, d2d(col(CA_PTT), st->ptt));
    HIPCHK(c, d2d(col(CA_LAM), st->lam));
  }
  nrto_status ls = launch_solve(c, warm ? 1 : 0, g);
  if (ls != NRTO_OK) return ls;
  HIPCHK(c, d2d(st->p, col(CA_P)));
  HIPCHK(c, d2d(st->pt, col(CA_PT)));
  HIPCHK(c, d2d(st->ptt, col(CA_PTT)));
  HIPCHK(c, d2d(st->lam, col(CA_LAM)));
  HIPCHK(c, d2d(st->pi, col(CA_PI)));
  if (rep) {
    HIPCHK(c, copy_out(rep, c->g.rep, (size_t)c->n, s));
    HIPCHK(c, hipStreamSynchronize(s));
    reports_to_us(c, rep, c->n);
  }
  return NRTO_OK;
}

// Copy a per-cone column of instance inst.
static hipError_t cone_col_out(nrto_ctx c, int inst, int col, double* dst) {
  const InstDev& d = c->hi[inst].d;
  return copy_out(dst, c->g.carr + (int64_t)col * c->ncones + d.cone0, (size_t)d.ng, c->stream);
}
static hipError_t cone_col_in(nrto_ctx c, int inst, int col, const double* src) {
  const InstDev& d = c->hi[inst].d;
  return copy_in(c->g.carr + (int64_t)col * c->ncones + d.cone0, src, (size_t)d.ng, c->stream);
}

extern "C" nrto_status nrto_get_solution(nrto_ctx c, int32_t inst, double* du, double* K, double* p, double* pt,
                                         double* pi, double* lam, double* mu) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (inst < 0 || inst >= c->n) return ctx_err(c, NRTO_ERR_ARG, "instance out of range");
  const InstDev& d = c->hi[inst].d;
  hipStream_t s = c->stream;
  HIPCHK(c, copy_out(du, c->g.du + d.oU, (size_t)d.T * d.nu, s));
  HIPCHK(c, copy_out(K, c->g.K + d.oK, (size_t)d.T * d.nu * d.nx, s));
  HIPCHK(c, cone_col_out(c, inst, CA_P, p));
  HIPCHK(c, cone_col_out(c, inst, CA_PT, pt));
  HIPCHK(c, cone_col_out(c, inst, CA_PI, pi));
  HIPCHK(c, cone_col_out(c, inst, CA_LAM, lam));
  HIPCHK(c, copy_out(mu, c->g.mu + inst, 1, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return NRTO_OK;
}

static nrto_status state_xfer(nrto_ctx c, int inst, double* st, double* nu, double* kt, double* ptt, bool out,
                              const double* ist, const double* inu, const double* ikt, const double* iptt) {
  const InstDev& d = c->hi[inst].d;
  hipStream_t s = c->stream;
  const size_t ne = (size_t)d.nent;
  if (c->opt.precision == NRTO_FP64) {
    double* dst = (double*)c->g.st + d.ent0;
    double* dnu = (double*)c->g.nu + d.ent0;
    if (out) {
      HIPCHK(c, copy_out(st, dst, ne, s));
      HIPCHK(c, copy_out(nu, dnu, ne, s));
    } else {
      HIPCHK(c, copy_in(dst, ist, ne, s));
      HIPCHK(c, copy_in(dnu, inu, ne, s));
    }
  } else {
    std::vector<float> f(ne);
    float* dst = (float*)c->g.st + d.ent0;
    float* dnu = (float*)c->g.nu + d.ent0;
    if (out) {
      if (st) {
        HIPCHK(c, copy_out(f.data(), dst, ne, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (size_t i = 0; i < ne; ++i) st[i] = f[i];
      }
      if (nu) {
        HIPCHK(c, copy_out(f.data(), dnu, ne, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (size_t i = 0; i < ne; ++i) nu[i] = f[i];
      }
    } else {
      if (ist) {
        for (size_t i = 0; i < ne; ++i) f[i] = (float)ist[i];
        HIPCHK(c, copy_in(dst, f.data(), ne, s));
        HIPCHK(c, hipStreamSynchronize(s));
      }
      if (inu) {
        for (size_t i = 0; i < ne; ++i) f[i] = (float)inu[i];
        HIPCHK(c, copy_in(dnu, f.data(), ne, s));
        HIPCHK(c, hipStreamSynchronize(s));
      }
    }
  }
  if (out) {
    HIPCHK(c, copy_out(kt, c->g.Kt + d.oK, (size_t)d.T * d.nu * d.nx, s));
    HIPCHK(c, cone_col_out(c, inst, CA_PTT, ptt));
  } else {
    HIPCHK(c, copy_in(c->g.Kt + d.oK, ikt, (size_t)d.T * d.nu * d.nx, s));
    HIPCHK(c, cone_col_in(c, inst, CA_PTT, iptt));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return NRTO_OK;
}

extern "C" nrto_status nrto_get_state(nrto_ctx c, int32_t inst, double* st, double* nu, double* kt, double* ptt) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (inst < 0 || inst >= c->n) return ctx_err(c, NRTO_ERR_ARG, "instance out of range");
  return state_xfer(c, inst, st, nu, kt, ptt, true, nullptr, nullptr, nullptr, nullptr);
}

extern "C" nrto_status nrto_set_state(nrto_ctx c, int32_t inst, const double* st, const double* nu,
                                      const double* kt, const double* ptt, const double* du, const double* K,
                                      const double* p, const double* pt, const double* lam) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (inst < 0 || inst >= c->n) return ctx_err(c, NRTO_ERR_ARG, "instance out of range");
  nrto_status s = state_xfer(c, inst, nullptr, nullptr, nullptr, nullptr, false, st, nu, kt, ptt);
  if (s != NRTO_OK) return s;
  const InstDev& d = c->hi[inst].d;
  hipStream_t sm = c->stream;
  HIPCHK(c, copy_in(c->g.du + d.oU, du, (size_t)d.T * d.nu, sm));
  HIPCHK(c, copy_in(c->g.K + d.oK, K, (size_t)d.T * d.nu * d.nx, sm));
  HIPCHK(c, cone_col_in(c, inst, CA_P, p));
  HIPCHK(c, cone_col_in(c, inst, CA_PT, pt));
  HIPCHK(c, cone_col_in(c, inst, CA_LAM, lam));
  // the (du, p) iterate's states follow from du; the solver recomputes them on its first Riccati pass
  int32_t zero = 0;
  HIPCHK(c, hipMemcpyAsync(c->g.flags + (int64_t)inst * 4, &zero, sizeof(int32_t), hipMemcpyHostToDevice, sm));
  HIPCHK(c, hipStreamSynchronize(sm));
  return NRTO_OK;
}

extern "C" nrto_status nrto_linearize(nrto_ctx c) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  int max_ng = 0;
  for (auto& h : c->hi) max_ng = std::max(max_ng, h.d.ng);
  HIPCHK(c, launch_linearize(c->g, c->n, max_ng, c->stream));
  return NRTO_OK;
}

extern "C" nrto_status nrto_get_nominal(nrto_ctx c, int32_t inst, double* uhat, double* K) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (inst < 0 || inst >= c->n) return ctx_err(c, NRTO_ERR_ARG, "instance out of range");
  const InstDev& d = c->hi[inst].d;
  HIPCHK(c, copy_out(uhat, c->g.uhat + d.oU, (size_t)d.T * d.nu, c->stream));
  HIPCHK(c, copy_out(K, c->g.K + d.oK, (size_t)d.T * d.nu * d.nx, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return NRTO_OK;
}


extern "C" nrto_status nrto_capture_step(nrto_ctx c, int32_t warm, int32_t with_linearize) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (!c->stream) return ctx_err(c, NRTO_ERR_ARG, "graph capture needs a non-default stream");
  if (c->opt.method == NRTO_FULLADMM || c->opt.precision == NRTO_FP32)
    return ctx_err(c, NRTO_ERR_STATE, "the FullADMM and FP32 device paths are switched off");
  if (c->step_exec) {
    HIPCHK(c, hipGraphExecDestroy(c->step_exec));
    c->step_exec = nullptr;
  }
  int max_ng = 0;
  for (auto& h : c->hi) max_ng = std::max(max_ng, h.d.ng);
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = with_linearize ? launch_linearize(c->g, c->n, max_ng, c->stream) : hipSuccess;
  nrto_status s = (e == hipSuccess) ? launch_solve(c, warm, c->g) : NRTO_ERR_HIP;
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
  if (e != hipSuccess) return ctx_err(c, NRTO_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
  if (s != NRTO_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e2 != hipSuccess) return ctx_err(c, NRTO_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
  e = hipGraphInstantiate(&c->step_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    c->step_exec = nullptr;
    return ctx_err(c, NRTO_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e));
  }
  return NRTO_OK;
}

extern "C" nrto_status nrto_launch_step(nrto_ctx c) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  if (!c->step_exec) return ctx_err(c, NRTO_ERR_STATE, "no captured step (call nrto_capture_step)");
  HIPCHK(c, hipGraphLaunch(c->step_exec, c->stream));
  return NRTO_OK;
}

extern "C" nrto_status nrto_get_reports(nrto_ctx c, nrto_solve_report* rep) {
  if (!c || !rep) return set_global_error(NRTO_ERR_ARG, "null argument");
  HIPCHK(c, copy_out(rep, c->g.rep, (size_t)c->n, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  reports_to_us(c, rep, c->n);
  return NRTO_OK;
}

extern "C" nrto_status nrto_scp_accept(nrto_ctx c, nrto_step_report* rep) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  std::vector<double> h(5 * (size_t)c->n);
  std::vector<nrto_solve_report> sr(c->n);
  hipError_t e = launch_scp_eval(c->g, c->n, 10.0, c->scp_out, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), c->scp_out, sizeof(double) * 5 * c->n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sr.data(), c->g.rep, sizeof(nrto_solve_report) * c->n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return ctx_err(c, NRTO_ERR_HIP, hipGetErrorString(e));
  if (rep)
    for (int i = 0; i < c->n; ++i) {
      rep[i].accepted = (int)h[5 * i];
      rep[i].status = sr[i].status;
      rep[i].merit_old = h[5 * i + 1];
      rep[i].merit_new = h[5 * i + 2];
      rep[i].predicted = h[5 * i + 3];
      rep[i].r_trust = h[5 * i + 4];
      rep[i].kkt = sr[i].kkt;
      rep[i].admm_iters = sr[i].admm_iters;
      rep[i].inner_iters = sr[i].inner_iters;
    }
  return NRTO_OK;
}

extern "C" nrto_status nrto_scp_step(nrto_ctx c, nrto_step_report* rep) {
  if (!c) return set_global_error(NRTO_ERR_ARG, "null context");
  nrto_status s = nrto_linearize(c);
  if (s != NRTO_OK) return s;
  // the KKT residual (and the robust margins the merit test reads) must be evaluated
  nrto_options keep = c->opt;
  if (!(c->opt.eps_kkt > 0.0)) c->opt.eps_kkt = 1e-300;
  s = nrto_solve_socp(c, 0, nullptr);
  c->opt = keep;
  if (s != NRTO_OK) return s;
  return nrto_scp_accept(c, rep);
}

extern "C" nrto_status nrto_warm_start(nrto_ctx c, const float* pred, int64_t ld, int32_t fallback_test,
                                       int32_t* accepted, double* residuals) {
  if (!c || !pred) return set_global_error(NRTO_ERR_ARG, "null argument");
  if (c->opt.method != NRTO_DR) return ctx_err(c, NRTO_ERR_STATE, "the learned warm start targets NRTO-DR");
  if (c->opt.precision == NRTO_FP32)
    return ctx_err(c, NRTO_ERR_STATE, "the FP32 solver path is switched off; use NRTO_FP64");
  if (fallback_test & ~3) return ctx_err(c, NRTO_ERR_ARG, "unknown warm-start flags");
  const bool gains = !(fallback_test & NRTO_WS_NO_GAINS);
  for (auto& h : c->hi)
    if (ld < (int64_t)h.d.T * h.d.nu * (gains ? h.d.nx + 1 : 1) + 2 * (int64_t)h.d.ng)
      return ctx_err(c, NRTO_ERR_ARG, "prediction row shorter than du (+ K) + p~ + pi");
  int32_t* acc = c->ws_acc;
  double* res = c->ws_res;
  SolveOpts o;
  fill_opts(c, o, 1);
  hipError_t e = hipSuccess;
  for (int gi = 0; gi < 3 && e == hipSuccess; ++gi) {
    const int cnt = c->group_off[gi + 1] - c->group_off[gi];
    e = launch_warm(c->g, o, c->group_nx[gi], c->order + c->group_off[gi], cnt, c->threads, c->smem, pred, ld,
                    fallback_test & 3, acc, res, c->stream);
  }
  if (e == hipSuccess && accepted) e = hipMemcpyAsync(accepted, acc, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && residuals) e = hipMemcpyAsync(residuals, res, sizeof(double) * 2 * c->n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return ctx_err(c, NRTO_ERR_HIP, hipGetErrorString(e));
  return NRTO_OK;
}
