// Persistent per-instance SOCP solver for gfx950: NRTO-DR and NRTO-FullADMM.
//
// One workgroup owns one instance for the whole solve (all ADMM and DR
// iterations, the (du, p) block and the KKT checks run inside one launch; no
// host round trip per iteration).  Per iteration the hot pass streams the cone
// entries once:
//   forward gain GEMM   eta_j[k] = r K_k' b_{j,k} + b_hat_j[k]  (K_k from LDS)
//   reflection / relaxation and the closed-form SOC projection (wave64
//   reductions: one wave per long cone, packed short cones per wave)
//   adjoint gain GEMM   R_k += b_{j,k} (.)'  accumulated with LDS atomics
// followed by the reduced-KKT block solve K_k = G_k^-1 R_k (FP64 Cholesky of
// the n_u x n_u blocks G_k, factored once per solve).  The (du, p) block is
// solved exactly by wave 0: semismooth Newton on the squared-hinge form whose
// Newton systems are LQ problems solved by a Riccati recursion, plus a
// trust-region multiplier search.
#include "common.hpp"
#include "internal.hpp"

namespace nrto {

constexpr int EMAX = 16;

// The workgroup's dynamic LDS (one instance's gains, adjoint accumulator,
// factors, reduction slots and (du, p) scratch).
extern __shared__ __align__(16) char nrto_dyn_smem[];
#ifndef NRTO_SOLVER_MAX_THREADS
#define NRTO_SOLVER_MAX_THREADS 512
#endif  // entries per lane of a long-cone task (cones up to 1024 entries)

template <typename F> __device__ __forceinline__ const F* bhat_ptr(const DevPtrs& g);
template <> __device__ __forceinline__ const double* bhat_ptr<double>(const DevPtrs& g) { return g.bhat64; }
template <> __device__ __forceinline__ const float* bhat_ptr<float>(const DevPtrs& g) { return g.bhat32; }
template <typename F> __device__ __forceinline__ const F* bvec_ptr(const DevPtrs& g);
template <> __device__ __forceinline__ const double* bvec_ptr<double>(const DevPtrs& g) { return g.bvec64; }
template <> __device__ __forceinline__ const float* bvec_ptr<float>(const DevPtrs& g) { return g.bvec32; }

__device__ __forceinline__ double atomic_load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Objects in global memory (device allocations) and in the workgroup's LDS.
// The pointers of an instance and of its LDS carve-up carry their address
// space in their type, so that functions the compiler keeps out of line
// still issue global and LDS instructions rather than flat ones (a flat load
// counts against both wait counters and so serialises LDS reads behind
// outstanding global loads).
// (The host pass of the compiler has no such address spaces; there the aliases
// are the plain types.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using G = __attribute__((address_space(1))) T;
template <typename T>
using L = __attribute__((address_space(3))) T;
#else
template <typename T>
using G = T;
template <typename T>
using L = T;
#endif

// Shared-memory carve-up for one instance workgroup.
template <typename F>
struct Smem {
  L<F>* Kf;        // NU*T*NX, u-major: Kf[(u*T + k)*NX + x]
  L<F>* Racc;      // NU*T*NX, same layout
  L<double>* Gl;   // T*NU*NU Cholesky factors
  L<double>* red;  // 128: [0, 64) block reductions, [64, 128) broadcast scalars
  L<double>* wscr; // W*128: per-wave cone sums / broadcast
  L<double>* qp;   // wave-0 QP scratch
  L<F>* bl;        // DR pass: per-wave block-vector slices, (T+1)*NU each (the LDS of qp, idle then)
  L<double>* gfb;  // Riccati feedback gains, T*NU*NX: [k][u][x] (the LDS of Kf when F is double)
  L<double>* gff;  // Riccati feedforward gains, T*NU: [k][u]
  L<int>* ctr;     // 4 ints
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t qp_scratch_doubles(int nx, int nu) {
  return 2 * nx * nx + nx + nx * nu + nu * nu + nu * nx + nu + 2 * nx + 64 +
         2 * (nx * nx + nx * nu + nu * (nx + 1)) + nu * (nx + 1) + nx * nx + nu * nu + nx + 160 + (2 * MAX_T + 4) / 2;
}

// The QP scratch block also holds the DR pass's per-wave block-vector slices.
__host__ __device__ inline size_t qp_region_bytes(int T, int nx, int nu, int fbytes, int W) {
  const size_t q = qp_scratch_doubles(nx, nu) * 8;
  const size_t b = (size_t)W * (T + 1) * nu * fbytes;
  return align16(q > b ? q : b);
}

__host__ __device__ inline size_t smem_bytes(int T, int nx, int nu, int fbytes, int W) {
  size_t s = 0;
  s += align16((size_t)nu * T * nx * fbytes);
  s += align16((size_t)nu * T * nx * fbytes);
  s += align16((size_t)T * nu * nu * 8);
  s += align16(128 * 8);
  s += align16((size_t)W * 128 * 8);
  s += qp_region_bytes(T, nx, nu, fbytes, W);
  s += align16((size_t)T * nu * 8);                  // feedforward gains
  if (fbytes < 8) s += align16((size_t)T * nu * nx * 8);   // feedback gains (else in Kf's LDS)
  s += 16;
  return s;
}

template <typename F>
__device__ Smem<F> carve(L<char>* base, int T, int nx, int nu, int W) {
  Smem<F> m;
  size_t o = 0;
  m.Kf = (L<F>*)(base + o); o += align16((size_t)nu * T * nx * sizeof(F));
  m.Racc = (L<F>*)(base + o); o += align16((size_t)nu * T * nx * sizeof(F));
  m.Gl = (L<double>*)(base + o); o += align16((size_t)T * nu * nu * 8);
  m.red = (L<double>*)(base + o); o += align16(128 * 8);
  m.wscr = (L<double>*)(base + o); o += align16((size_t)W * 128 * 8);
  m.qp = (L<double>*)(base + o); o += qp_region_bytes(T, nx, nu, (int)sizeof(F), W);
  m.bl = (L<F>*)m.qp;
  m.gff = (L<double>*)(base + o); o += align16((size_t)T * nu * 8);
  if (sizeof(F) < 8) {
    m.gfb = (L<double>*)(base + o);
    o += align16((size_t)T * nu * nx * 8);
  } else {
    // Kf is dead while the (du, p) block runs: the next DR K-solve rewrites
    // all of it before it is read again, and the KKT residual reads K from
    // global memory
    m.gfb = (L<double>*)m.Kf;
  }
  m.ctr = (L<int>*)(base + o);
  return m;
}

// Block-wide sum of up to 4 values per thread (deterministic order).
template <int NV>
__device__ void block_sum(double* red, double (&v)[NV], int W) {
  static_assert(NV >= 1 && NV <= 8, "up to 8 values (8 waves x 8 slots of the 64 reduction slots)");
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane_id() == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave_id() * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int w = 0; w < W; ++w) s += red[w * NV + i];
    v[i] = s;
  }
  __syncthreads();
}

template <int NV>
__device__ void block_max(double* red, double (&v)[NV], int W) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_max(v[i]);
  __syncthreads();
  if (lane_id() == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave_id() * 4 + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = red[i];
    for (int w = 1; w < W; ++w) s = fmax(s, red[w * 4 + i]);
    v[i] = s;
  }
  __syncthreads();
}

// 1/sqrt(s) for a normal s > 0: the hardware estimate (relative error below
// 2^-24, measured) refined by two Newton-Raphson steps for the reciprocal
// square root, y <- y + y (1 - s y^2) / 2, each of which squares the relative
// error.  Measured over 2^20 values from 1e-300 to 1e300: within 1.3 units in
// the last place of the exact value, and within 2 of a correctly rounded sqrt
// followed by a correctly rounded division, which takes several times as long.
__device__ __forceinline__ double rsqrt_nr(double s) {
  double y = __builtin_amdgcn_rsq(s);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(s * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

template <int NU>
__device__ __forceinline__ void chol_inplace(double* G) {
  // lower Cholesky factor L of an NU x NU SPD matrix stored row-major, with
  // 1 / L_jj stored on the diagonal (the solves multiply by it: one division
  // per column instead of one per entry); upper part untouched
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    double s = G[j * NU + j];
#pragma unroll
    for (int l = 0; l < j; ++l) s -= G[j * NU + l] * G[j * NU + l];
    const double rd = rsqrt_nr(fmax(s, 1e-300));
    G[j * NU + j] = rd;
#pragma unroll
    for (int i = j + 1; i < NU; ++i) {
      double t = G[i * NU + j];
#pragma unroll
      for (int l = 0; l < j; ++l) t -= G[i * NU + l] * G[j * NU + l];
      G[i * NU + j] = t * rd;
    }
  }
}

// Solve (L L') z = z in place with a factor from chol_inplace.
template <int NU>
__device__ __forceinline__ void chol_solve(const double* L, double (&z)[NU]) {
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    double t = z[i];
#pragma unroll
    for (int l = 0; l < i; ++l) t -= L[i * NU + l] * z[l];
    z[i] = t * L[i * NU + i];
  }
#pragma unroll
  for (int i = NU - 1; i >= 0; --i) {
    double t = z[i];
#pragma unroll
    for (int l = i + 1; l < NU; ++l) t -= L[l * NU + i] * z[l];
    z[i] = t * L[i * NU + i];
  }
}

// One FP64 matrix-core product on a wave: D = A B + C with A 16x4, B 4x16, C and
// D 16x16.  Lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; register i of
// lane l holds C[l / 16 + 4 i][l % 16], and so D.
typedef double f64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f64x4 mfma_f64_16x16x4(double a, double b, f64x4 c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
#else
  (void)a;
  (void)b;
  return c;
#endif
}

// ----------------------------------------------------------------------------
// Instance view: pointers of one instance.
template <int NX, int NU, typename F>
struct Inst {
  int T, ng, nent, ntask;
  double r, r_trust;
  const G<int32_t>* cm;
  G<double>* ca;        // carr + cone0; column stride = ncones
  int64_t cstride;
  const G<double>* W;
  const G<F>* bhat;
  const G<F>* bvec;
  G<F>* st;
  G<F>* nuv;
  const G<double> *A, *B, *xhat, *uhat;
  G<double> *dx, *du, *dx2, *du2, *K, *Kt, *kscr;
  const G<double> *Q, *Ru, *RK2, *xg;
  const G<int32_t>* tls;  // state cones by time: [tls[t], tls[t+1])
  const G<int32_t>* tlc;  // control cones by step: [tlc[k], tlc[k+1])
  const G<WaveTask>* tasks;
  const G<uint64_t>* tmask;
  const G<LaneBlock>* lblock;   // lane table of the packed tasks (tasks nlong, nlong + 1, ...)
  int nlong;
  G<double>* mu;
  G<double>* iscr;
  G<int32_t>* flags;

  __device__ G<double>& C(int a, int j) const { return ca[(int64_t)a * cstride + j]; }
};

// Wave-uniform copy of a value held in vector registers or on the stack of an
// out-of-line function (every lane holds the same value).  In scalar registers
// the compiler keeps such pointers live instead of reloading them from the
// argument block on the stack inside loops: a stack reload is a vector-memory
// load, and waiting for it also waits for every global load issued before it
// (the prefetches of the next stage).
// Value of lane l (wave-uniform l) of a double in every lane.
__device__ __forceinline__ double lane_read(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename P>
__device__ __forceinline__ P uni(P p) {
  if constexpr (sizeof(P) == 8) {
    const uint64_t v = __builtin_bit_cast(uint64_t, p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return __builtin_bit_cast(P, ((uint64_t)hi << 32) | lo);
  } else {
    static_assert(sizeof(P) == 4, "32- or 64-bit values");
    return __builtin_bit_cast(P, (uint32_t)__builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, p)));
  }
}

// Raw buffer view of one array of an instance (wave-uniform base and size in a
// buffer descriptor).  A load addresses it by a vector offset (here always the
// lane's fixed offset, a register the loop never rewrites) plus a scalar
// offset; offsets at or past the end read 0.  Used for the prefetches of the
// Riccati sweep, whose loads must stay in flight while the wave reuses its
// other registers.
template <typename T>
struct Buf {
#if defined(__HIP_DEVICE_COMPILE__)
  __amdgpu_buffer_rsrc_t r;
#else
  const T* p;
#endif
  // n elements of T starting at p (n * sizeof(T) < 2^31)
  __device__ static Buf make(const G<T>* p, int64_t n) {
    Buf b;
#if defined(__HIP_DEVICE_COMPILE__)
    // word 3 of a raw (untyped) buffer descriptor on the gfx9 family
    b.r = __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n * (int64_t)sizeof(T)), 0x00020000);
#else
    b.p = p;
    (void)n;
#endif
    return b;
  }
  // element at byte offset voff + soff
  __device__ T ld(uint32_t voff, uint32_t soff) const {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(T) == 8)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
#else
    return *(const T*)((const char*)p + voff + soff);
#endif
  }
  // elements at byte offsets voff + soff and voff + soff + 8 (one 16-byte load)
  __device__ void ld2(uint32_t voff, uint32_t soff, T& v0, T& v1) const {
#if defined(__HIP_DEVICE_COMPILE__)
    static_assert(sizeof(T) == 8, "64-bit elements");
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    v0 = __builtin_bit_cast(T, (u32x2){w[0], w[1]});
    v1 = __builtin_bit_cast(T, (u32x2){w[2], w[3]});
#else
    v0 = *(const T*)((const char*)p + voff + soff);
    v1 = *(const T*)((const char*)p + voff + soff + 8);
#endif
  }
  // store v at byte offset voff + soff; an offset past the n elements stores
  // nothing (the buffer's range check), so lanes can opt out without a branch
  __device__ void st(uint32_t voff, uint32_t soff, T v) const {
#if defined(__HIP_DEVICE_COMPILE__)
    static_assert(sizeof(T) == 8, "64-bit elements");
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
#else
    *(T*)((char*)p + voff + soff) = v;
#endif
  }
};

// The instance view with every member made wave-uniform (see uni).
template <int NX, int NU, typename F>
__device__ __forceinline__ Inst<NX, NU, F> uniform_inst(const Inst<NX, NU, F>& I) {
  Inst<NX, NU, F> U;
  U.T = uni(I.T);
  U.ng = uni(I.ng);
  U.nent = uni(I.nent);
  U.ntask = uni(I.ntask);
  U.r = uni(I.r);
  U.r_trust = uni(I.r_trust);
  U.cm = uni(I.cm);
  U.ca = uni(I.ca);
  U.cstride = uni(I.cstride);
  U.W = uni(I.W);
  U.bhat = uni(I.bhat);
  U.bvec = uni(I.bvec);
  U.st = uni(I.st);
  U.nuv = uni(I.nuv);
  U.A = uni(I.A);
  U.B = uni(I.B);
  U.xhat = uni(I.xhat);
  U.uhat = uni(I.uhat);
  U.dx = uni(I.dx);
  U.du = uni(I.du);
  U.dx2 = uni(I.dx2);
  U.du2 = uni(I.du2);
  U.K = uni(I.K);
  U.Kt = uni(I.Kt);
  U.kscr = uni(I.kscr);
  U.Q = uni(I.Q);
  U.Ru = uni(I.Ru);
  U.RK2 = uni(I.RK2);
  U.xg = uni(I.xg);
  U.tls = uni(I.tls);
  U.tlc = uni(I.tlc);
  U.tasks = uni(I.tasks);
  U.tmask = uni(I.tmask);
  U.lblock = uni(I.lblock);
  U.nlong = uni(I.nlong);
  U.mu = uni(I.mu);
  U.iscr = uni(I.iscr);
  U.flags = uni(I.flags);
  return U;
}

template <int NX, int NU, typename F>
__device__ Inst<NX, NU, F> make_inst(const DevPtrs& g, int ii) {
  const InstDev& d = g.inst[ii];
  Inst<NX, NU, F> I;
  I.T = d.T;
  I.ng = d.ng;
  I.nent = d.nent;
  I.ntask = d.ntask;
  I.r = d.radius;
  I.r_trust = d.r_trust;
  I.cm = (const G<int32_t>*)(g.cmeta + d.cone0 * CM_N);
  I.ca = (G<double>*)(g.carr + d.cone0);
  I.cstride = g.ncones;
  I.W = (const G<double>*)(g.w + d.oW);
  I.bhat = (const G<F>*)(bhat_ptr<F>(g) + d.ent0);
  I.bvec = (const G<F>*)(bvec_ptr<F>(g) + d.bv0);
  I.st = (G<F>*)((F*)g.st + d.ent0);
  I.nuv = (G<F>*)((F*)g.nu + d.ent0);
  I.A = (const G<double>*)(g.A + d.oA);
  I.B = (const G<double>*)(g.B + d.oB);
  I.xhat = (const G<double>*)(g.xhat + d.oX);
  I.uhat = (const G<double>*)(g.uhat + d.oU);
  I.dx = (G<double>*)(g.dx + d.oX);
  I.du = (G<double>*)(g.du + d.oU);
  I.dx2 = (G<double>*)(g.dx2 + d.oX);
  I.du2 = (G<double>*)(g.du2 + d.oU);
  I.K = (G<double>*)(g.K + d.oK);
  I.Kt = (G<double>*)(g.Kt + d.oK);
  I.kscr = (G<double>*)(g.kscr + d.oK);
  const double* prm = g.prm + d.oP;
  ParamOffsets po = param_offsets(NX, NU, d.n_obs);
  I.Q = (const G<double>*)(prm + po.Q);
  I.Ru = (const G<double>*)(prm + po.Ru);
  I.RK2 = (const G<double>*)(prm + po.RK2);
  I.xg = (const G<double>*)(prm + po.xg);
  I.tls = (const G<int32_t>*)(g.tl + d.oTL);
  I.tlc = I.tls + (d.T + 2);
  I.tasks = (const G<WaveTask>*)(g.tasks + d.task0);
  I.tmask = (const G<uint64_t>*)(g.tmask + d.task0);
  I.lblock = (const G<LaneBlock>*)(g.lblock + d.lb0 * 64);
  I.nlong = d.nlong;
  I.mu = (G<double>*)(g.mu + ii);
  I.iscr = (G<double>*)(g.iscr + (int64_t)ii * ISCR_N);
  I.flags = (G<int32_t>*)(g.flags + (int64_t)ii * 4);
  return I;
}

// Linear part a_j(du, dx) of constraint j: w_j' dx_{t_j} (state) or s du_{k,i} (control).
template <int NX, int NU, typename F>
__device__ __forceinline__ double cons_lin(const Inst<NX, NU, F>& I, int j, const double* dx, const double* du) {
  const int32_t* m = I.cm + j * CM_N;
  if (m[CM_KIND] == 0) {
    const double* w = I.W + (int64_t)j * NX;
    const double* x = dx + (int64_t)m[CM_TIME] * NX;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NX; ++i) s += w[i] * x[i];
    return s;
  }
  return (double)m[CM_CSIGN] * du[(int64_t)m[CM_TIME] * NU + m[CM_CIDX]];
}

// ----------------------------------------------------------------------------
// Factor: G_k = 2 RK2 + shift I + coef sum_j b_jk b_jk'  -> Cholesky in LDS.
template <int NX, int NU, typename F>
__device__ void factor_blocks(const Inst<NX, NU, F>& I, Smem<F>& S, double coef, double shift) {
  const int T = I.T;
  for (int i = threadIdx.x; i < T * NU * NU; i += blockDim.x) S.Gl[i] = 0.0;
  __syncthreads();
  for (int j = threadIdx.x; j < I.ng; j += blockDim.x) {
    const int32_t* m = I.cm + j * CM_N;
    const int k0 = m[CM_K0], nb = m[CM_NBLK], bo = m[CM_BOFF];
    for (int b = 0; b < nb; ++b) {
      if (k0 + b >= T) break;
      const F* bv = I.bvec + (int64_t)(bo + b) * NU;
      double v[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) v[u] = (double)bv[u];
      double* G = S.Gl + (k0 + b) * NU * NU;
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int w = 0; w <= u; ++w)
          if (v[u] * v[w] != 0.0) atomicAdd(&G[u * NU + w], v[u] * v[w]);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < T; k += blockDim.x) {
    double* G = S.Gl + k * NU * NU;
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
      for (int w = 0; w <= u; ++w)
        G[u * NU + w] = coef * G[u * NU + w] + 2.0 * I.RK2[u * NU + w] + (u == w ? shift : 0.0);
    chol_inplace<NU>(G);
  }
  __syncthreads();
}

// K-solve.  DR: K = G^-1 (sigma_chi K~ + sigma_s r Racc), K~ += alpha (K - K~).
// FullADMM: K = G'^-1 (2 RK2 K + rho r Racc).  Racc is zeroed; Kf mirrors K.
template <int NX, int NU, typename F, int METHOD>
__device__ void k_solve(const Inst<NX, NU, F>& I, Smem<F>& S, const SolveOpts& o, double sig,
                        double (&kacc)[2]) {
  const int T = I.T;
  for (int col = threadIdx.x; col < T * NX; col += blockDim.x) {
    const int k = col / NX, x = col - k * NX;
    double z[NU];
    if (METHOD == NRTO_DR) {
      const double a = sig * I.r;
#pragma unroll
      for (int u = 0; u < NU; ++u)
        z[u] = o.sigma_chi * I.Kt[(k * NU + u) * NX + x] + a * (double)S.Racc[(u * T + k) * NX + x];
    } else {
      const double a = o.rho * I.r;
      double kp[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) kp[u] = I.K[(k * NU + u) * NX + x];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NU; ++w) s += I.RK2[u * NU + w] * kp[w];
        z[u] = 2.0 * s + a * (double)S.Racc[(u * T + k) * NX + x];
      }
    }
    chol_solve<NU>(S.Gl + k * NU * NU, z);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      I.K[(k * NU + u) * NX + x] = z[u];
      S.Kf[(u * T + k) * NX + x] = (F)z[u];
      S.Racc[(u * T + k) * NX + x] = (F)0;
      if (METHOD == NRTO_DR) {
        double kt = I.Kt[(k * NU + u) * NX + x];
        I.Kt[(k * NU + u) * NX + x] = kt + o.alpha * (z[u] - kt);
        kacc[0] += (z[u] - kt) * (z[u] - kt);
        kacc[1] += z[u] * z[u];
      }
    }
  }
  __syncthreads();
}

// Load K (double, global) into Kf and zero Racc.
template <int NX, int NU, typename F>
__device__ void load_kf(const Inst<NX, NU, F>& I, Smem<F>& S) {
  const int T = I.T;
  for (int i = threadIdx.x; i < T * NU * NX; i += blockDim.x) {
    const int k = i / (NU * NX), rem = i - k * NU * NX, u = rem / NX, x = rem - u * NX;
    S.Kf[(u * T + k) * NX + x] = (F)I.K[i];
    S.Racc[(u * T + k) * NX + x] = (F)0;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// Task iteration helpers.
__device__ __forceinline__ int next_task(int* ctr) {
  int t = 0;
  if (lane_id() == 0) t = atomicAdd(ctr, 1);
  return __shfl(t, 0, NRTO_WAVE);
}

// Per-entry geometry of an eta entry: block time k, component x, block index.
template <int NX>
__device__ __forceinline__ void entry_block(const int32_t* m, int le, int& k, int& x, int& b) {
  const int m1 = le - 1;
  const int blk = m1 / NX;
  x = m1 - blk * NX;
  k = m[CM_K0] + blk;
  b = m[CM_BOFF] + blk;
}

template <int NX, int NU, typename F>
__device__ __forceinline__ F fwd_gemm(const Inst<NX, NU, F>& I, const Smem<F>& S, int T, int k, int x,
                                      const F* bv) {
  F f = (F)0;
  if (k >= T) return f;   // last block of a state constraint at t = T: b = 0, no gain
#pragma unroll
  for (int u = 0; u < NU; ++u) f += bv[u] * S.Kf[(u * T + k) * NX + x];
  return f;
}

template <int NX, int NU, typename F>
__device__ __forceinline__ void adj_gemm(Smem<F>& S, int T, int k, int x, const F* bv, F v) {
  if (k >= T) return;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const F c = bv[u] * v;
    if (c != (F)0) atomicAdd(&S.Racc[(u * T + k) * NX + x], c);
  }
}

// Closed-form projection scale: returns (t_hat, eta scale) for input (t, a = ||eta||).
__device__ __forceinline__ void soc_case(double t, double a, double& that, double& scale) {
  if (a <= t) {
    that = t;
    scale = 1.0;
  } else if (a <= -t) {
    that = 0.0;
    scale = 0.0;
  } else {
    that = 0.5 * (t + a);
    scale = that / a;
  }
}

// ----------------------------------------------------------------------------
// DR pass: one relaxed DR iteration over all cones of the instance (after the
// K-solve).  Accumulates sum ||delta s~||^2 and ||s~||^2.
//
// A long cone (more than 64 entries) is handled by one wave.  The wave first
// copies the cone's block vectors b_{j,k} (at most (T+1)*NU values) into its
// LDS slice, and every lane issues the loads of its entries of s~ and b_hat
// (independent, so they are in flight together with the block vectors).  It
// then forms eta(K) from the block vectors and K_k in LDS, reduces the
// reflected norm, and projects / relaxes / stores its entries.  Up to 64*E
// entries (E = 2, 4, 8 or 12, by the cone's length; see dr_stage) a lane keeps s~,
// b_hat and eta of its E entries in registers (one sweep over the cone's data);
// longer cones take two sweeps (the second reloads s~ and b_hat).  The cone's first block, first block vector and multiplier
// data come with the task.
// Chunks of 64 entries a lane holds in one sweep, at most: 12 where the DR pass
// then still compiles without register spills (n_x = 12, n_u = 4), else 8.
template <int NX, int NU>
constexpr int dr_stage() {
  return (NX == 12 && NU == 4) ? 12 : 8;
}

// The cone's multiplier data (cd: p~~, p, lambda of the cone, loaded with the
// cone's entries) enter the t slot: p~ = (sigma_chi p~~ + rho p + lambda +
// sigma_s s~_0) / den.
struct ConeDual {
  double ptt, p, lam;
};

// Copy of a cone's n block-vector values into the wave's LDS slice, 4*64 values
// a round: load() issues a round's loads, store() writes them to LDS.  The
// first round is loaded before the cone's entries and stored after them (the
// store then waits for these loads only: vector-memory loads complete in
// order); cones with more than 256 values (long horizons) take further rounds.
template <typename F>
struct BlockStage {
  static constexpr int PL = 4;
  F v[PL];
  __device__ void load(const G<F>* __restrict__ bv, int n, int base) {
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int idx = base + lane_id() + i * NRTO_WAVE;
      v[i] = (idx < n) ? bv[idx] : (F)0;
    }
  }
  __device__ void store(F* bl, int n, int base) const {
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int idx = base + lane_id() + i * NRTO_WAVE;
      if (idx < n) bl[idx] = v[i];
    }
  }
  // the rounds after the first
  __device__ void rest(const G<F>* __restrict__ bv, int n, F* bl) {
    for (int base = PL * NRTO_WAVE; base < n; base += PL * NRTO_WAVE) {
      load(bv, n, base);
      store(bl, n, base);
    }
  }
};

// eta entry (before the reflection) of entry le >= 1 of a cone starting at block k0:
// r * b_{j,k}' K_k[:, x] + b_hat (a block at k = T, the terminal block of a state
// constraint, carries no gain).
template <int NX, int NU, typename F>
__device__ __forceinline__ F cone_eta(const F* bl, const F* Kf, int T, int k0, int le, F r, F bh, int& k, int& x,
                                      int& blk) {
  const int q = le - 1;
  blk = q / NX;
  x = q - blk * NX;
  k = k0 + blk;
  F f = (F)0;
  if (k < T) {
#pragma unroll
    for (int u = 0; u < NU; ++u) f += bl[blk * NU + u] * Kf[(u * T + k) * NX + x];
  }
  return r * f + bh;
}

template <int NX, int NU, typename F>
__device__ __forceinline__ void cone_adjoint(const F* bl, F* Racc, int T, int k, int x, int blk, F d) {
  if (k >= T) return;
#pragma unroll
  for (int u = 0; u < NU; ++u) atomicAdd(&Racc[(u * T + k) * NX + x], bl[blk * NU + u] * d);
}

// One sweep: a cone of at most 64*E entries.
template <int NX, int NU, typename F, int E>
__device__ __forceinline__ void dr_long_cone(const WaveTask tk, G<F>* __restrict__ st, const G<F>* __restrict__ bhat,
                                             const G<F>* __restrict__ bvec, const F* Kf, F* Racc, F* bl, int T, F r,
                                             double al, const ConeDual cd, double chi, double rho, double sig,
                                             double den, G<double>* ca_pt, G<double>* ca_ptt, double (&acc)[5]) {
  const int lane = lane_id();
  const int len = tk.len;
  const int k0 = tk.k0;
  const G<F>* bvp = bvec + (int64_t)tk.boff * NU;
  const int nbv = ((len - 1) / NX) * NU;
  BlockStage<F> bs;
  bs.load(bvp, nbv, 0);
  F stv[E], bhv[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int le = lane + i * NRTO_WAVE;
    stv[i] = (le < len) ? st[le] : (F)0;
    bhv[i] = (le >= 1 && le < len) ? bhat[le] : (F)0;
  }
  bs.store(bl, nbv, 0);
  bs.rest(bvp, nbv, bl);
  wave_sync();   // the block vectors in LDS
  // forward gain GEMM and the norm of the reflected eta
  F sv[E];
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int le = lane + i * NRTO_WAVE;
    sv[i] = (F)0;
    if (le >= 1 && le < len) {
      int k, x, blk;
      sv[i] = cone_eta<NX, NU, F>(bl, Kf, T, k0, le, r, bhv[i], k, x, blk);
      const F sr = (F)2 * sv[i] - stv[i];
      sq += (double)sr * (double)sr;
    }
  }
  double ptc = 0.0, tr0 = 0.0;
  if (lane == 0) {
    ptc = (chi * cd.ptt + rho * cd.p + cd.lam + sig * (double)stv[0]) / den;
    tr0 = (double)((F)2 * (F)ptc - stv[0]);
  }
  const double a = sqrt(wave_sum(sq));
  const double tref = lane_read(tr0, 0);
  double that, scale;
  soc_case(tref, a, that, scale);
  double dsum = 0.0, nsum = 0.0, ssum = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int le = lane + i * NRTO_WAVE;
    if (le < len) {
      F s, shat;
      if (le == 0) {
        s = (F)ptc;
        shat = (F)that;
      } else {
        s = sv[i];
        const F sr = (F)2 * s - stv[i];
        shat = (F)(scale * (double)sr);
      }
      const F diff = shat - s;
      const F stn = stv[i] + (F)al * diff;
      st[le] = stn;
      const double dd = al * (double)diff;
      dsum += dd * dd;
      nsum += (double)stn * (double)stn;
      ssum += (double)s * (double)s;
      if (le > 0) {
        const int q = le - 1, blk = q / NX, x = q - blk * NX;
        cone_adjoint<NX, NU, F>(bl, Racc, T, k0 + blk, x, blk, stn - bhv[i]);
      }
    }
  }
  if (lane == 0) {
    *ca_pt = ptc;
    *ca_ptt = cd.ptt + al * (ptc - cd.ptt);
  }
  acc[0] += dsum;
  acc[1] += nsum;
  acc[4] += ssum;
  wave_sync();   // the slice is reused by the wave's next cone
}

// Cones longer than one sweep holds: two sweeps over the entries in groups of
// E chunks (the first forms the reflected norm, the second reloads the group,
// recomputes eta, projects, relaxes and accumulates the adjoint).
template <int NX, int NU, typename F, int E>
__device__ __forceinline__ void dr_long_cone_2pass(const WaveTask tk, G<F>* __restrict__ st,
                                                   const G<F>* __restrict__ bhat, const G<F>* __restrict__ bvec,
                                                   const F* Kf, F* Racc, F* bl, int T, F r, double al,
                                                   const ConeDual cd, double chi, double rho, double sig, double den,
                                                   G<double>* ca_pt, G<double>* ca_ptt, double (&acc)[5]) {
  const int lane = lane_id();
  const int len = tk.len;
  const int k0 = tk.k0;
  const G<F>* bvp = bvec + (int64_t)tk.boff * NU;
  const int nbv = ((len - 1) / NX) * NU;
  BlockStage<F> bs;
  bs.load(bvp, nbv, 0);
  const F st0 = (lane == 0) ? st[0] : (F)0;   // used after the first sweep
  double sq = 0.0;
  for (int base = 0; base < len; base += E * NRTO_WAVE) {
    F stv[E], bhv[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int le = base + lane + i * NRTO_WAVE;
      const bool in = le >= 1 && le < len;
      stv[i] = in ? st[le] : (F)0;
      bhv[i] = in ? bhat[le] : (F)0;
    }
    if (base == 0) {
      bs.store(bl, nbv, 0);
      bs.rest(bvp, nbv, bl);
    }
    wave_sync();   // the block vectors in LDS
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int le = base + lane + i * NRTO_WAVE;
      if (le >= 1 && le < len) {
        int k, x, blk;
        const F sr = (F)2 * cone_eta<NX, NU, F>(bl, Kf, T, k0, le, r, bhv[i], k, x, blk) - stv[i];
        sq += (double)sr * (double)sr;
      }
    }
  }
  double ptc = 0.0, tr0 = 0.0;
  if (lane == 0) {
    ptc = (chi * cd.ptt + rho * cd.p + cd.lam + sig * (double)st0) / den;
    tr0 = (double)((F)2 * (F)ptc - st0);
  }
  const double a = sqrt(wave_sum(sq));
  const double tref = lane_read(tr0, 0);
  double that, scale;
  soc_case(tref, a, that, scale);
  double dsum = 0.0, nsum = 0.0, ssum = 0.0;
  for (int base = 0; base < len; base += E * NRTO_WAVE) {
    F stv[E], bhv[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int le = base + lane + i * NRTO_WAVE;
      stv[i] = (le < len) ? st[le] : (F)0;
      bhv[i] = (le >= 1 && le < len) ? bhat[le] : (F)0;
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int le = base + lane + i * NRTO_WAVE;
      if (le < len) {
        F s, shat;
        int k = 0, x = 0, blk = 0;
        if (le == 0) {
          s = (F)ptc;
          shat = (F)that;
        } else {
          s = cone_eta<NX, NU, F>(bl, Kf, T, k0, le, r, bhv[i], k, x, blk);
          shat = (F)(scale * (double)((F)2 * s - stv[i]));
        }
        const F diff = shat - s;
        const F stn = stv[i] + (F)al * diff;
        st[le] = stn;
        const double dd = al * (double)diff;
        dsum += dd * dd;
        nsum += (double)stn * (double)stn;
        ssum += (double)s * (double)s;
        if (le > 0) cone_adjoint<NX, NU, F>(bl, Racc, T, k, x, blk, stn - bhv[i]);
      }
    }
  }
  if (lane == 0) {
    *ca_pt = ptc;
    *ca_ptt = cd.ptt + al * (ptc - cd.ptt);
  }
  acc[0] += dsum;
  acc[1] += nsum;
  acc[4] += ssum;
  wave_sync();   // the slice is reused by the wave's next cone
}

// Arguments of the DR pass, passed by value to a separately compiled function
// so that its register allocation does not compete with the rest of the solve.
template <typename F>
struct DrArgs {
  const WaveTask* tasks;
  const uint64_t* tmask;
  const LaneBlock* lblock;
  const int32_t* cm;
  double* ca;          // per-cone columns, column stride cstride
  int64_t cstride;
  F* st;
  const F* bhat;
  const F* bvec;
  const F* Kf;
  F* Racc;
  F* bl;               // per-wave block-vector slices
  double* wscr;
  int* ctr;
  int64_t lds_ctr_off;   // byte offset of ctr in the dynamic LDS
  int T, ntask, nlong;
  double r, al, sigma_chi, rho, sig;
};

struct Acc5 {
  double v[5];
};

// A function compiled on its own only sees generic pointers in its arguments:
// the DR pass re-derives their address spaces (G<T>: global memory; as_lds: the
// workgroup's dynamic LDS) so that it issues global and LDS instructions
// instead of flat ones.
template <typename T>
__device__ __forceinline__ T* as_lds(const void* p, const char* base) {
  return (T*)(nrto_dyn_smem + ((const char*)p - base));
}

template <int NX, int NU, typename F>
__device__ __noinline__ Acc5 dr_pass_impl(DrArgs<F> g) {
  {
    const char* base = (const char*)g.ctr - g.lds_ctr_off;
    g.Kf = as_lds<F>(g.Kf, base);
    g.Racc = as_lds<F>(g.Racc, base);
    g.bl = as_lds<F>(g.bl, base);
    g.wscr = as_lds<double>(g.wscr, base);
    g.ctr = as_lds<int>(g.ctr, base);
  }
  const G<WaveTask>* tasks = (const G<WaveTask>*)g.tasks;
  const G<uint64_t>* tmask = (const G<uint64_t>*)g.tmask;
  const G<LaneBlock>* lblock = (const G<LaneBlock>*)g.lblock;
  G<double>* ca = (G<double>*)g.ca;
  G<F>* gst = (G<F>*)g.st;
  const G<F>* gbhat = (const G<F>*)g.bhat;
  const G<F>* gbvec = (const G<F>*)g.bvec;
  Acc5 out;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int T = g.T;
  const int lane = lane_id();
  const F r = (F)g.r;
  const double al = g.al;
  const double den = g.rho + g.sigma_chi + g.sig;
  const double rho = g.rho, sig = g.sig;
  double* ws = g.wscr + wave_id() * 128;
  F* bl = g.bl + wave_id() * (T + 1) * NU;
  auto C = [&](int col, int j) -> G<double>& { return ca[(int64_t)col * g.cstride + j]; };
  // Static schedule: wave w takes tasks w, w + W, w + 2W, ... of the list (long
  // cones first, by decreasing length).  A wave's next task is known in
  // advance, so its descriptor is loaded while the current task is processed;
  // a long cone's first block and block-vector offset come with the
  // descriptor, and its multiplier data are loaded with its entries.
  const int W = (int)(blockDim.x / NRTO_WAVE);
  constexpr int DRS = dr_stage<NX, NU>();
  // (a packed task's lane-table row follows from its index: the packed tasks
  // come after the g.nlong long ones, so its load is issued with the descriptor)
  auto load_task = [&](int t, WaveTask& k, uint64_t& mask, LaneBlock& lb) {
    const G<WaveTask>* p = tasks + t;
    k.cone = p->cone;
    k.ncone = p->ncone;
    k.ebeg = p->ebeg;
    k.len = p->len;
    k.k0 = p->k0;
    k.boff = p->boff;
    mask = tmask[t];
    if (t >= g.nlong) {
      const G<LaneBlock>* q = lblock + (int64_t)(t - g.nlong) * NRTO_WAVE + lane;
      lb.k = q->k;
      lb.b = q->b;
    }
  };
  int t = uni((int)wave_id());
  WaveTask tk = {0, 0, 0, 0, 0, 0, 0, 0};
  uint64_t tkmask = 0;
  LaneBlock tklb = {-1, -1};
  if (t < g.ntask) load_task(t, tk, tkmask, tklb);
  for (; t < g.ntask; t += W) {
    WaveTask tkn = tk;
    uint64_t tknmask = 0;
    LaneBlock tknlb = {-1, -1};
    if (t + W < g.ntask) load_task(t + W, tkn, tknmask, tknlb);
    if (tk.ncone == 1 && tk.len > NRTO_WAVE) {
      const int c = tk.cone;
      const ConeDual cd = {C(CA_PTT, c), C(CA_P, c), C(CA_LAM, c)};
      G<F>* st = gst + tk.ebeg;
      const G<F>* bh = gbhat + tk.ebeg;
      G<double>* cpt = &C(CA_PT, c);
      G<double>* cptt = &C(CA_PTT, c);
      if (tk.len <= 2 * NRTO_WAVE)
        dr_long_cone<NX, NU, F, 2>(tk, st, bh, gbvec, g.Kf, g.Racc, bl, T, r, al, cd, g.sigma_chi, rho, sig, den,
                                   cpt, cptt, acc);
      else if (tk.len <= 4 * NRTO_WAVE)
        dr_long_cone<NX, NU, F, 4>(tk, st, bh, gbvec, g.Kf, g.Racc, bl, T, r, al, cd, g.sigma_chi, rho, sig, den,
                                   cpt, cptt, acc);
      else if (tk.len <= 8 * NRTO_WAVE)
        dr_long_cone<NX, NU, F, 8>(tk, st, bh, gbvec, g.Kf, g.Racc, bl, T, r, al, cd, g.sigma_chi, rho, sig, den,
                                   cpt, cptt, acc);
      else if (DRS > 8 && tk.len <= DRS * NRTO_WAVE)
        dr_long_cone<NX, NU, F, DRS>(tk, st, bh, gbvec, g.Kf, g.Racc, bl, T, r, al, cd, g.sigma_chi, rho, sig, den,
                                     cpt, cptt, acc);
      else
        dr_long_cone_2pass<NX, NU, F, DRS>(tk, st, bh, gbvec, g.Kf, g.Racc, bl, T, r, al, cd, g.sigma_chi, rho, sig,
                                           den, cpt, cptt, acc);
    } else {
      // packed short cones: one entry per lane; its block time and block vector
      // come from the lane table, its cone (for the t slot) from the mask
      const uint64_t mask = tkmask;
      const int l = lane;
      const bool valid = l < tk.len;
      const uint64_t pre = mask & ((l == 63) ? ~0ull : ((2ull << l) - 1ull));
      const int cl = __popcll(pre) - 1;
      const int cs = 63 - __clzll(pre);
      const int le = l - cs;
      const int c = tk.cone + cl;
      ws[l] = 0.0;
      wave_sync();
      F s = (F)0, stv = (F)0, bh = (F)0;
      F bvr[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) bvr[u] = (F)0;
      double ptc = 0.0;
      int k = 0, x = 0;
      bool has_gain = false;
      if (valid) {
        const int64_t e = tk.ebeg + l;
        stv = gst[e];
        if (le == 0) {
          ptc = (g.sigma_chi * C(CA_PTT, c) + rho * C(CA_P, c) + C(CA_LAM, c) + sig * (double)stv) / den;
          s = (F)ptc;
          ws[64 + cl] = (double)((F)2 * s - stv);
        } else {
          x = (le - 1) % NX;
          k = tklb.k;
          bh = gbhat[e];
          F f = (F)0;
          if (k >= 0) {
            has_gain = true;
            const G<F>* bv = gbvec + (int64_t)tklb.b * NU;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
              bvr[u] = bv[u];
              f += bvr[u] * g.Kf[(u * T + k) * NX + x];
            }
          }
          s = r * f + bh;
          const F sr = (F)2 * s - stv;
          atomicAdd(&ws[cl], (double)sr * (double)sr);
        }
      }
      wave_sync();
      if (valid) {
        const int64_t e = tk.ebeg + l;
        const double a = sqrt(ws[cl]);
        const double tref = ws[64 + cl];
        double that, scale;
        soc_case(tref, a, that, scale);
        const F sr = (F)2 * s - stv;
        const F shat = (le == 0) ? (F)that : (F)(scale * (double)sr);
        const F diff = shat - s;
        const F stn = stv + (F)al * diff;
        gst[e] = stn;
        const double dd = al * (double)diff;
        acc[0] += dd * dd;
        acc[1] += (double)stn * (double)stn;
        acc[4] += (double)s * (double)s;
        if (le == 0) {
          C(CA_PT, c) = ptc;
          const double pt0 = C(CA_PTT, c);
          C(CA_PTT, c) = pt0 + al * (ptc - pt0);
        } else if (has_gain) {
          const F d = stn - bh;
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const F cu = bvr[u] * d;
            if (cu != (F)0) atomicAdd(&g.Racc[(u * T + k) * NX + x], cu);
          }
        }
      }
      wave_sync();
    }
    tk = tkn;
    tkmask = tknmask;
    tklb = tknlb;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) out.v[i] = acc[i];
  return out;
}

template <int NX, int NU, typename F>
__device__ __forceinline__ void dr_pass(const Inst<NX, NU, F>& I, Smem<F>& S, const SolveOpts& o, double rho,
                                        double sig, double (&acc)[5]) {
  DrArgs<F> g;
  g.tasks = I.tasks;
  g.tmask = I.tmask;
  g.lblock = I.lblock;
  g.cm = I.cm;
  g.ca = I.ca;
  g.cstride = I.cstride;
  g.st = I.st;
  g.bhat = I.bhat;
  g.bvec = I.bvec;
  g.Kf = S.Kf;
  g.Racc = S.Racc;
  g.bl = S.bl;
  g.wscr = S.wscr;
  g.ctr = S.ctr;
  g.lds_ctr_off = (int64_t)((const char*)S.ctr - (const char*)nrto_dyn_smem);
  g.T = I.T;
  g.ntask = I.ntask;
  g.nlong = I.nlong;
  g.r = I.r;
  g.al = o.alpha;
  g.sigma_chi = o.sigma_chi;
  g.rho = rho;
  g.sig = sig;
  const Acc5 a = dr_pass_impl<NX, NU, F>(g);
#pragma unroll
  for (int i = 0; i < 5; ++i) acc[i] += a.v[i];
}

// R pass: Racc = sum_j b_jk (s~_eta - b_hat)' from the current DR state.
template <int NX, int NU, typename F>
__device__ void r_pass(const Inst<NX, NU, F>& I, Smem<F>& S) {
  const int T = I.T;
  for (int t = next_task(S.ctr); t < I.ntask; t = next_task(S.ctr)) {
    const WaveTask tk = I.tasks[t];
    // lane -> entries of the task; the cone of each entry by scanning cone offsets
    int c = tk.cone;
    for (int le0 = lane_id(); le0 < tk.len; le0 += NRTO_WAVE) {
      const int eloc = tk.ebeg + le0;
      while (c + 1 < tk.cone + tk.ncone && I.cm[(c + 1) * CM_N + CM_EOFF] <= eloc) ++c;
      const int32_t* m = I.cm + c * CM_N;
      const int le = eloc - m[CM_EOFF];
      if (le == 0) continue;
      int k, x, b;
      entry_block<NX>(m, le, k, x, b);
      adj_gemm<NX, NU, F>(S, T, k, x, I.bvec + (int64_t)b * NU, I.st[eloc] - I.bhat[eloc]);
    }
  }
}

// FullADMM pass: (deferred) lambda_nu update with the current K, Block 1
// projection, adjoint accumulation of nu - b_hat.  acc: [r_nu^2 (previous
// iteration), r_d^2 / rho^2].
template <int NX, int NU, typename F>
__device__ void fa_pass(const Inst<NX, NU, F>& I, Smem<F>& S, const SolveOpts& o, bool pending,
                        double (&acc)[2]) {
  const int T = I.T;
  const int lane = lane_id();
  const F r = (F)I.r;
  double* ws = S.wscr + wave_id() * 128;
  for (int t = next_task(S.ctr); t < I.ntask; t = next_task(S.ctr)) {
    const WaveTask tk = I.tasks[t];
    if (tk.ncone == 1 && tk.len > NRTO_WAVE) {
      const int c = tk.cone;
      const int32_t* m = I.cm + c * CM_N;
      F yv[EMAX], lv[EMAX];
      double sq = 0.0, rn = 0.0, yt = 0.0;
#pragma unroll
      for (int i = 0; i < EMAX; ++i) {
        const int le = lane + i * NRTO_WAVE;
        yv[i] = lv[i] = (F)0;
        if (le < tk.len) {
          const int64_t e = tk.ebeg + le;
          if (le == 0) {
            yt = I.C(CA_P, c) + I.C(CA_LAM, c);
            yv[i] = (F)yt;
          } else {
            int k, x, b;
            entry_block<NX>(m, le, k, x, b);
            const F a = r * fwd_gemm<NX, NU, F>(I, S, T, k, x, I.bvec + (int64_t)b * NU) + I.bhat[e];
            F l = I.st[e];
            if (pending) {
              const F dn = a - I.nuv[e];
              l += dn;
              rn += (double)dn * (double)dn;
            }
            lv[i] = l;
            yv[i] = a + l;
            sq += (double)yv[i] * (double)yv[i];
          }
        }
      }
      const double an = sqrt(wave_sum(sq));
      const double tref = __shfl((double)yv[0], 0, NRTO_WAVE);
      double that, scale;
      soc_case(tref, an, that, scale);
#pragma unroll
      for (int i = 0; i < EMAX; ++i) {
        const int le = lane + i * NRTO_WAVE;
        if (le < tk.len) {
          const int64_t e = tk.ebeg + le;
          if (le == 0) {
            const double old = I.C(CA_PT, c);
            acc[1] += (that - old) * (that - old);
            I.C(CA_PT, c) = that;
          } else {
            const F nv = (F)(scale * (double)yv[i]);
            I.st[e] = lv[i];
            I.nuv[e] = nv;
            int k, x, b;
            entry_block<NX>(m, le, k, x, b);
            adj_gemm<NX, NU, F>(S, T, k, x, I.bvec + (int64_t)b * NU, nv - I.bhat[e]);
          }
        }
      }
      acc[0] += rn;
    } else {
      const uint64_t mask = I.tmask[t];
      const int l = lane;
      const bool valid = l < tk.len;
      const uint64_t pre = mask & ((l == 63) ? ~0ull : ((2ull << l) - 1ull));
      const int cl = __popcll(pre) - 1;
      const int cs = 63 - __clzll(pre);
      const int le = l - cs;
      const int c = tk.cone + cl;
      ws[l] = 0.0;
      wave_sync();
      F y = (F)0, lvv = (F)0;
      int k = 0, x = 0, b = 0;
      const int32_t* m = I.cm + c * CM_N;
      if (valid) {
        const int64_t e = tk.ebeg + l;
        if (le == 0) {
          const double yt = I.C(CA_P, c) + I.C(CA_LAM, c);
          y = (F)yt;
          ws[64 + cl] = yt;
        } else {
          entry_block<NX>(m, le, k, x, b);
          const F a = r * fwd_gemm<NX, NU, F>(I, S, T, k, x, I.bvec + (int64_t)b * NU) + I.bhat[e];
          lvv = I.st[e];
          if (pending) {
            const F dn = a - I.nuv[e];
            lvv += dn;
            acc[0] += (double)dn * (double)dn;
          }
          y = a + lvv;
          atomicAdd(&ws[cl], (double)y * (double)y);
        }
      }
      wave_sync();
      if (valid) {
        const int64_t e = tk.ebeg + l;
        double that, scale;
        soc_case(ws[64 + cl], sqrt(ws[cl]), that, scale);
        if (le == 0) {
          const double old = I.C(CA_PT, c);
          acc[1] += (that - old) * (that - old);
          I.C(CA_PT, c) = that;
        } else {
          const F nv = (F)(scale * (double)y);
          I.st[e] = lvv;
          I.nuv[e] = nv;
          adj_gemm<NX, NU, F>(S, T, k, x, I.bvec + (int64_t)b * NU, nv - I.bhat[e]);
        }
      }
      wave_sync();
    }
  }
}

// Commit the deferred FullADMM dual update lambda_nu += A_hat k_v + b_hat - nu.
template <int NX, int NU, typename F>
__device__ void fa_commit(const Inst<NX, NU, F>& I, Smem<F>& S) {
  const int T = I.T;
  const F r = (F)I.r;
  for (int t = next_task(S.ctr); t < I.ntask; t = next_task(S.ctr)) {
    const WaveTask tk = I.tasks[t];
    int c = tk.cone;
    for (int le0 = lane_id(); le0 < tk.len; le0 += NRTO_WAVE) {
      const int eloc = tk.ebeg + le0;
      while (c + 1 < tk.cone + tk.ncone && I.cm[(c + 1) * CM_N + CM_EOFF] <= eloc) ++c;
      const int32_t* m = I.cm + c * CM_N;
      const int le = eloc - m[CM_EOFF];
      if (le == 0) continue;
      int k, x, b;
      entry_block<NX>(m, le, k, x, b);
      const F a = r * fwd_gemm<NX, NU, F>(I, S, T, k, x, I.bvec + (int64_t)b * NU) + I.bhat[eloc];
      I.st[eloc] = I.st[eloc] + (a - I.nuv[eloc]);
    }
  }
}

// ----------------------------------------------------------------------------
// (du, p) block on wave 0.
template <int NX, int NU>
struct QPScratch {
  L<double> *V, *v, *PA, *PB, *Huu, *Hux, *hu, *tmp, *red;
  L<double>* AB;      // double buffer of one stage's data for the backward pass, halves of
                      // AB_N doubles: A (NX*NX), B (NX*NU), then x_k, u_k
  static constexpr int AB_N = NX * NX + NX * NU + NU * (NX + 1);
  // half (k & 1) of the double buffer (address arithmetic: an array of two
  // pointers indexed at run time would live on the stack)
  __device__ L<double>* ab(int k) const { return AB + (k & 1) * AB_N; }
  L<double>* G;       // gains of the current stage, NU*(NX+1)
  L<double> *Qs, *Rs, *xg;   // LDS copies of Q, Ru, the goal state
  L<double>* act;     // active state cones of a stage: 64 int indices, 64 betas, 64 gradient values
  L<double>* tl;      // LDS copy of the stage lists: state cones by time (T + 2 ints), control
                      // cones by step (T + 1 ints)
  L<double>* gfb;     // gains of all stages: feedback [k][u][x] (T*NU*NX) and
  L<double>* gff;     // feedforward [k][u] (T*NU), outside the scratch block
};

template <int NX, int NU>
__device__ QPScratch<NX, NU> qp_carve(L<double>* q, L<double>* gfb, L<double>* gff) {
  QPScratch<NX, NU> s;
  s.gfb = gfb;
  s.gff = gff;
  s.V = q; q += NX * NX;
  s.v = q; q += NX;
  s.PA = q; q += NX * NX;
  s.PB = q; q += NX * NU;
  s.Huu = q; q += NU * NU;
  s.Hux = q; q += NU * NX;
  s.hu = q; q += NU;
  s.tmp = q; q += 2 * NX;
  s.red = q; q += 64;
  s.AB = q; q += 2 * QPScratch<NX, NU>::AB_N;
  s.G = q; q += NU * (NX + 1);
  s.Qs = q; q += NX * NX;
  s.Rs = q; q += NU * NU;
  s.xg = q; q += NX;
  s.act = q; q += 160;
  s.tl = q;
  return s;
}

// Active-set flags of one stage, loaded a stage ahead: lane l holds the flag and
// beta of state cone tls[t] + l, and the flag, beta, input index and sign of
// control cone tlc[k] + l (cones beyond the first 64 of a stage are read
// directly when used).  load() only issues the loads: the loaded values are
// first used a stage later (a use right after the load would wait for it, and
// with it for every global load issued earlier, such as the stage prefetch).
struct StageFlags {
  int s0, s1, c0, c1;
  // raw loaded values (lanes past the stage's cones hold whatever follows in
  // the arrays; the accessors mask them)
  double sact, sbeta;          // state cone: flag, beta
  double cact, cbeta;          // control cone: flag, beta
  int ccidx, ccsign;           // control cone: input index, bound sign
  __device__ bool sf() const { return lane_id() < s1 - s0 && sact != 0.0; }
  __device__ bool cf() const { return lane_id() < c1 - c0 && cact != 0.0; }
  __device__ double cbs() const { return cbeta * (double)ccsign; }   // beta times the bound's sign (lanes with cf())
  // bact, bbeta: the instance's CA_ACT and CA_BETA columns; bcm: its cone metadata
  __device__ void load(const Buf<double>& bact, const Buf<double>& bbeta, const Buf<int32_t>& bcm,
                       const L<int>* tls, const L<int>* tlc, int t, int k) {
    // the list bounds are wave-uniform (scalar registers): each load below is
    // a scalar offset plus the lane's fixed offset
    s0 = uni(tls[t]);
    s1 = uni(tls[t + 1]);
    const uint32_t l = (uint32_t)lane_id();
    sact = bact.ld(l * 8u, (uint32_t)s0 * 8u);
    sbeta = bbeta.ld(l * 8u, (uint32_t)s0 * 8u);
    if (k >= 0) {
      c0 = uni(tlc[k]);
      c1 = uni(tlc[k + 1]);
    } else {
      c0 = c1 = 0;
    }
    cact = bact.ld(l * 8u, (uint32_t)c0 * 8u);
    cbeta = bbeta.ld(l * 8u, (uint32_t)c0 * 8u);
    ccidx = bcm.ld(l * (uint32_t)(CM_N * 4) + CM_CIDX * 4u, (uint32_t)c0 * (uint32_t)(CM_N * 4));
    ccsign = bcm.ld(l * (uint32_t)(CM_N * 4) + CM_CSIGN * 4u, (uint32_t)c0 * (uint32_t)(CM_N * 4));
  }
};

// Add the active state-constraint terms of time t to (V, v): rho w w', rho beta w.
// The active cones of a stage are compacted into an LDS list and their
// gradient rows gathered in batches of 64 / NX (one load round trip per batch)
// into a 64-double LDS buffer.
template <int NX, int NU, typename F>
__device__ void add_state_terms(const Inst<NX, NU, F>& I, QPScratch<NX, NU>& q, const StageFlags& fl, double rho) {
  const int lane = lane_id();
  constexpr int PERB = NRTO_WAVE / NX;
  int* act_c = (int*)q.act;
  double* act_b = q.act + 32;
  double* wb = q.act + 96;
  for (int base = fl.s0; base < fl.s1; base += NRTO_WAVE) {
    bool f;
    double bl;
    if (base == fl.s0) {
      f = fl.sf();
      bl = fl.sbeta;
    } else {
      f = (base + lane < fl.s1) && I.C(CA_ACT, base + lane) != 0.0;
      bl = f ? I.C(CA_BETA, base + lane) : 0.0;
    }
    const uint64_t mask = __ballot(f);
    const int nact = __popcll(mask);
    if (nact == 0) continue;
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    if (f) {
      act_c[rank] = base + lane;
      act_b[rank] = bl;
    }
    wave_sync();
    for (int b0 = 0; b0 < nact; b0 += PERB) {
      const int na = min(PERB, nact - b0);
      const int a = lane / NX, i = lane - a * NX;
      if (a < na) wb[a * NX + i] = I.W[(int64_t)act_c[b0 + a] * NX + i];
      wave_sync();
      for (int idx = lane; idx < NX * NX; idx += NRTO_WAVE) {
        const int r = idx / NX, c = idx - r * NX;
        double sum = 0.0;
        for (int aa = 0; aa < na; ++aa) sum += wb[aa * NX + r] * wb[aa * NX + c];
        q.V[idx] += rho * sum;
      }
      if (lane < NX) {
        double sum = 0.0;
        for (int aa = 0; aa < na; ++aa) sum += act_b[b0 + aa] * wb[aa * NX + lane];
        q.v[lane] += rho * sum;
      }
      wave_sync();
    }
  }
}

// Stage data of the backward Riccati pass: A_k (NX*NX), B_k (NX*NU), the
// nominal x_k (NX) and u_k (NU), staged in LDS one stage ahead (each lane holds
// its share of the next stage in registers while the current one is computed).
// Each array is read lane-strided from its own (wave-uniform) base, so that a
// load's address is a scalar base plus the lane's fixed offset: the address
// registers are never overwritten while the loads are in flight.
template <int N>
struct LanePrefetch {
  static constexpr int PER = (N + NRTO_WAVE - 1) / NRTO_WAVE;
  double v[PER];
  // elements [first, first + N) of the array behind b (lanes past N read
  // whatever follows, or 0 past the array's end; store() drops them)
  __device__ void load(const Buf<double>& b, int first) {
    const uint32_t lo = (uint32_t)lane_id() * 8u;
#pragma unroll
    for (int i = 0; i < PER; ++i) v[i] = b.ld(lo + (uint32_t)(i * NRTO_WAVE * 8), (uint32_t)first * 8u);
  }
  __device__ void store(double* dst) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = lane_id() + i * NRTO_WAVE;
      if (idx < N) dst[idx] = v[i];
    }
  }
};

template <int NX, int NU>
struct StagePrefetch {
  static constexpr int NA = NX * NX, NB = NX * NU;
  LanePrefetch<NA> a;
  LanePrefetch<NB> b;
  LanePrefetch<NX> x;
  LanePrefetch<NU> u;
  // stage k of the arrays A, B, x_hat, u_hat
  __device__ void load(const Buf<double>& bA, const Buf<double>& bB, const Buf<double>& bx, const Buf<double>& bu,
                       int k) {
    a.load(bA, k * NA);
    b.load(bB, k * NB);
    x.load(bx, k * NX);
    u.load(bu, k * NU);
  }
  __device__ void store(double* dst) const {
    a.store(dst);
    b.store(dst + NA);
    x.store(dst + NA + NB);
    u.store(dst + NA + NB + NX);
  }
};

// Riccati solve of the LQ problem of the current active set at multiplier mu;
// result in (du2, dx2).  Compiled out of line (one copy, its own register
// allocation) with the instance view and LDS carve-up by value.
template <int NX, int NU, typename F>
__device__ __noinline__ void riccati(const Inst<NX, NU, F> Iarg, QPScratch<NX, NU> qarg, double rho, double mu) {
  const Inst<NX, NU, F> I = uniform_inst(Iarg);
  QPScratch<NX, NU> q = qp_carve<NX, NU>(uni(qarg.V), uni(qarg.gfb), uni(qarg.gff));   // V is the carve-up's base
  const int lane = lane_id();
  // stage products on the matrix cores when [A | B] fits one 16-wide tile
  constexpr int NXU = NX + NU;
  constexpr bool MFMA_STAGE = NXU <= 16 && NU <= 4;
  constexpr int KB = (NX + 3) / 4;   // 4-deep blocks of the contraction over n_x
  const int T = I.T;
  StagePrefetch<NX, NU> pf;
  StageFlags fl, fln;
  const Buf<double> bA = Buf<double>::make(I.A, (int64_t)T * NX * NX);
  const Buf<double> bB = Buf<double>::make(I.B, (int64_t)T * NX * NU);
  const Buf<double> bx = Buf<double>::make(I.xhat, (int64_t)(T + 1) * NX);
  const Buf<double> bu = Buf<double>::make(I.uhat, (int64_t)T * NU);
  const Buf<double> bact = Buf<double>::make(&I.C(CA_ACT, 0), I.ng);
  const Buf<double> bbeta = Buf<double>::make(&I.C(CA_BETA, 0), I.ng);
  const Buf<int32_t> bcm = Buf<int32_t>::make(I.cm, (int64_t)I.ng * CM_N);
  auto stage_load = [&](int k) { pf.load(bA, bB, bx, bu, k); };
  stage_load(T - 1);
  const L<int>* tls = (const L<int>*)q.tl;
  const L<int>* tlc = tls + (T + 2);
  fl.load(bact, bbeta, bcm, tls, tlc, T, -1);
  fln.load(bact, bbeta, bcm, tls, tlc, T - 1, T - 1);
  // LDS copies of the stage-invariant cost data
  for (int idx = lane; idx < NX * NX; idx += NRTO_WAVE) q.Qs[idx] = I.Q[idx];
  for (int idx = lane; idx < NU * NU; idx += NRTO_WAVE) q.Rs[idx] = I.Ru[idx];
  if (lane < NX) {
    q.xg[lane] = I.xg[lane];
    q.tmp[lane] = I.xhat[T * NX + lane];
  }
  wave_sync();
  // terminal cost-to-go
  for (int idx = lane; idx < NX * NX; idx += NRTO_WAVE) {
    const int i = idx / NX, j = idx - i * NX;
    q.V[idx] = 2.0 * q.Qs[idx] + (i == j ? mu : 0.0);
  }
  if (lane < NX) {
    double s = 0.0;
    for (int j = 0; j < NX; ++j) s += q.Qs[lane * NX + j] * (q.tmp[j] - q.xg[j]);
    q.v[lane] = 2.0 * s;
  }
  pf.store(q.ab(T - 1));
  wave_sync();
  add_state_terms<NX, NU, F>(I, q, fl, rho);
  wave_sync();
  // no vector-memory load is outstanding when the stage loop starts: the
  // compiler then tracks only the loads the loop issues itself, and the loads
  // of the next stage stay in flight while the current one is computed
  // (immediate: vmcnt 0, expcnt and lgkmcnt unconstrained)
  __builtin_amdgcn_s_waitcnt(0x0F70);
  for (int k = T - 1; k >= 0; --k) {
    const double* A = q.ab(k);
    const double* B = A + NX * NX;
    const double* xk = B + NX * NU;
    const double* uk = xk + NX;
    fl = fln;
    if (k > 0) {
      stage_load(k - 1);
      fln.load(bact, bbeta, bcm, tls, tlc, k - 1, k - 1);
    }
    // stage products.  Matrix cores (n_x + n_u <= 16, n_u <= 4): with
    // C = [A | B], P = V C (three 16x16x4 products for n_x = 12) and then
    // M = C' P; register kb of P is the B operand of block kb of the second
    // product and the A operand is C's value the lane already loaded.  M holds
    // A'V A (kept in registers for the cost-to-go), H_ux = B'V A and B'V B.
    [[maybe_unused]] f64x4 Mreg = {0.0, 0.0, 0.0, 0.0};
    if constexpr (MFMA_STAGE) {
      const int r = lane & 15, kq = lane >> 4;
      f64x4 P = {0.0, 0.0, 0.0, 0.0};
      double cv[KB];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int kk = 4 * kb + kq;
        const double va = (r < NX && kk < NX) ? q.V[r * NX + kk] : 0.0;
        cv[kb] = (kk < NX && r < NXU) ? (r < NX ? A[kk * NX + r] : B[kk * NU + (r - NX)]) : 0.0;
        P = mfma_f64_16x16x4(va, cv[kb], P);
      }
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) Mreg = mfma_f64_16x16x4(cv[kb], P[kb], Mreg);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = kq + 4 * i;
        if (row >= NX && row < NXU) {
          const int u = row - NX;
          if (r < NX) q.Hux[u * NX + r] = Mreg[i];
          else if (r < NXU) q.Huu[u * NU + (r - NX)] = 2.0 * q.Rs[u * NU + (r - NX)] + Mreg[i];
        }
      }
    } else {
#pragma unroll 1
      for (int idx = lane; idx < NX * NX; idx += NRTO_WAVE) {
        const int i = idx / NX, j = idx - i * NX;
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) s += q.V[i * NX + l] * A[l * NX + j];
        q.PA[idx] = s;
      }
#pragma unroll 1
      for (int idx = lane; idx < NX * NU; idx += NRTO_WAVE) {
        const int i = idx / NU, u = idx - i * NU;
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) s += q.V[i * NX + l] * B[l * NU + u];
        q.PB[idx] = s;
      }
      wave_sync();
#pragma unroll 1
      for (int idx = lane; idx < NU * NU; idx += NRTO_WAVE) {
        const int u = idx / NU, w = idx - u * NU;
        double s = 2.0 * q.Rs[idx];
#pragma unroll
        for (int i = 0; i < NX; ++i) s += B[i * NU + u] * q.PB[i * NU + w];
        q.Huu[idx] = s;
      }
#pragma unroll 1
      for (int idx = lane; idx < NU * NX; idx += NRTO_WAVE) {
        const int u = idx / NX, j = idx - u * NX;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NX; ++i) s += B[i * NU + u] * q.PA[i * NX + j];
        q.Hux[idx] = s;
      }
    }
    if (lane < NU) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NU; ++w) s += q.Rs[lane * NU + w] * uk[w];
      s *= 2.0;
#pragma unroll
      for (int i = 0; i < NX; ++i) s += B[i * NU + lane] * q.v[i];
      q.hu[lane] = s;
    }
    wave_sync();
    {
      // gains of stage k: every lane factors H_uu (plus rho on the diagonal of
      // the active control bounds, whose flags, beta * sign and input index were
      // prefetched a stage ahead by the lane of each cone) in registers, and
      // lanes 0..NX solve one right-hand side each (the columns of H_ux, then h_u)
      double Hl[NU * NU], hl[NU];
#pragma unroll
      for (int i = 0; i < NU * NU; ++i) Hl[i] = q.Huu[i];
#pragma unroll
      for (int u = 0; u < NU; ++u) hl[u] = q.hu[u];
      uint64_t cmask = __ballot(fl.cf());
      while (cmask) {
        const int bit = __ffsll((unsigned long long)cmask) - 1;
        cmask &= cmask - 1;
        const int ci = __builtin_amdgcn_readlane(fl.ccidx, bit);   // bit is wave-uniform
        const double hb = lane_read(fl.cbs(), bit);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if (u == ci) {
            Hl[u * NU + u] += rho;
            hl[u] += rho * hb;
          }
        }
      }
      for (int c = fl.c0 + NRTO_WAVE; c < fl.c1; ++c) {   // control cones beyond the first 64
        if (I.C(CA_ACT, c) == 0.0) continue;
        const int ci = I.cm[c * CM_N + CM_CIDX];
        const double hb = I.C(CA_BETA, c) * (double)I.cm[c * CM_N + CM_CSIGN];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if (u == ci) {
            Hl[u * NU + u] += rho;
            hl[u] += rho * hb;
          }
        }
      }
      chol_inplace<NU>(Hl);
      if (lane <= NX) {
        double z[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) z[u] = (lane < NX) ? q.Hux[u * NX + lane] : hl[u];
        chol_solve<NU>(Hl, z);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if (lane < NX) q.gfb[(k * NU + u) * NX + lane] = -z[u];
          else q.gff[k * NU + u] = -z[u];
          q.G[u * (NX + 1) + lane] = -z[u];
        }
      }
    }
    wave_sync();
    if (k > 0 && MFMA_STAGE) {
      // cost-to-go of stage k: V = 2Q + mu I + A'V A + H_ux' G_x, the last term
      // one more matrix-core product accumulated onto A'V A; the upper triangle
      // is written to both halves (V is symmetric)
      const int r = lane & 15, kq = lane >> 4;
      const double ha = (kq < NU && r < NX) ? q.Hux[kq * NX + r] : 0.0;
      const double gb = (kq < NU && r < NX) ? q.G[kq * (NX + 1) + r] : 0.0;
      const f64x4 D = mfma_f64_16x16x4(ha, gb, Mreg);
      double vv = 0.0;
      if (lane < NX) {
        double sum = 0.0;
        for (int j = 0; j < NX; ++j) sum += q.Qs[lane * NX + j] * (xk[j] - q.xg[j]);
        sum *= 2.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) sum += A[l * NX + lane] * q.v[l];
#pragma unroll
        for (int u = 0; u < NU; ++u) sum += q.Hux[u * NX + lane] * q.G[u * (NX + 1) + NX];
        vv = sum;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = kq + 4 * i;
        if (row < NX && r < NX && row <= r) {
          const double val = 2.0 * q.Qs[row * NX + r] + (row == r ? mu : 0.0) + D[i];
          q.V[row * NX + r] = val;
          q.V[r * NX + row] = val;
        }
      }
      wave_sync();
      if (lane < NX) q.v[lane] = vv;
      pf.store(q.ab(k - 1));
      wave_sync();
      add_state_terms<NX, NU, F>(I, q, fl, rho);
      wave_sync();
    } else if (k > 0) {
      // cost-to-go of stage k: V = 2Q + mu I + A'(V A) + H_ux' G_x is symmetric;
      // its upper triangle is computed and written to both halves
      constexpr int NTRI = NX * (NX + 1) / 2;
      constexpr int NPER = (NTRI + NRTO_WAVE - 1) / NRTO_WAVE;
      double nv[NPER];
      int ti[NPER], tj[NPER];
#pragma unroll
      for (int n = 0; n < NPER; ++n) {
        const int idx = lane + n * NRTO_WAVE;
        nv[n] = 0.0;
        ti[n] = tj[n] = 0;
        if (idx >= NTRI) continue;
        int i = 0, rem = idx;   // row i of the upper triangle holds NX - i entries
        while (rem >= NX - i) {
          rem -= NX - i;
          ++i;
        }
        const int j = i + rem;
        double sum = 2.0 * q.Qs[i * NX + j] + (i == j ? mu : 0.0);
#pragma unroll
        for (int l = 0; l < NX; ++l) sum += A[l * NX + i] * q.PA[l * NX + j];
#pragma unroll
        for (int u = 0; u < NU; ++u) sum += q.Hux[u * NX + i] * q.G[u * (NX + 1) + j];
        nv[n] = sum;
        ti[n] = i;
        tj[n] = j;
      }
      double vv = 0.0;
      if (lane < NX) {
        double sum = 0.0;
        for (int j = 0; j < NX; ++j) sum += q.Qs[lane * NX + j] * (xk[j] - q.xg[j]);
        sum *= 2.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) sum += A[l * NX + lane] * q.v[l];
#pragma unroll
        for (int u = 0; u < NU; ++u) sum += q.Hux[u * NX + lane] * q.G[u * (NX + 1) + NX];
        vv = sum;
      }
      // V, v are not read by the products above (only V A, H_ux and G): update in place
#pragma unroll
      for (int n = 0; n < NPER; ++n) {
        if (lane + n * NRTO_WAVE >= NTRI) continue;
        q.V[ti[n] * NX + tj[n]] = nv[n];
        q.V[tj[n] * NX + ti[n]] = nv[n];
      }
      wave_sync();
      if (lane < NX) q.v[lane] = vv;
      pf.store(q.ab(k - 1));
      wave_sync();
      add_state_terms<NX, NU, F>(I, q, fl, rho);
      wave_sync();
    }
  }
  // forward rollout from dx_0 = 0, u_k = G_k x_k + g_k, x_{k+1} = A_k x_k + B_k u_k.
  // The state (lanes 0..NX-1) and the control (lanes 0..NU-1) stay in registers
  // and are read across lanes; lane i < NX holds row i of A_k and B_k in
  // registers, loaded FD stages ahead (register sets picked at compile time: the
  // stage loop is unrolled by FD); the gains are read from LDS.  Loads and the
  // stores of (du2, dx2) are issued without branches (lanes without a row or an
  // element use an offset past the end, which the buffer's range check turns
  // into a zero load or a dropped store; stages past T-1 reload stage T-1), so
  // that the compiler's wait counts keep FD stages in flight.
  constexpr int FD = 4;
  constexpr uint32_t OOR = 0x7FFFFFF0u;   // byte offset past any array here
  const Buf<double> bdu2 = Buf<double>::make(I.du2, (int64_t)T * NU);
  const Buf<double> bdx2 = Buf<double>::make(I.dx2, (int64_t)(T + 1) * NX);
  const uint32_t vra = lane < NX ? (uint32_t)(lane * NX) * 8u : OOR;
  const uint32_t vrb = lane < NX ? (uint32_t)(lane * NU) * 8u : OOR;
  double ar[FD][NX], br[FD][NU];
  auto row_load = [&](double (&a)[NX], double (&b)[NU], int k) {   // 16-byte loads
    const int kk = k < T ? k : T - 1;
    const uint32_t sa = (uint32_t)(kk * NX * NX) * 8u, sb = (uint32_t)(kk * NX * NU) * 8u;
#pragma unroll
    for (int j = 0; j + 1 < NX; j += 2) bA.ld2(vra + (uint32_t)j * 8u, sa, a[j], a[j + 1]);
    if constexpr (NX % 2) a[NX - 1] = bA.ld(vra + (uint32_t)(NX - 1) * 8u, sa);
#pragma unroll
    for (int u = 0; u + 1 < NU; u += 2) bB.ld2(vrb + (uint32_t)u * 8u, sb, b[u], b[u + 1]);
    if constexpr (NU % 2) b[NU - 1] = bB.ld(vrb + (uint32_t)(NU - 1) * 8u, sb);
  };
#pragma unroll
  for (int d = 0; d < FD; ++d) row_load(ar[d], br[d], d);
  bdx2.st(lane < NX ? (uint32_t)lane * 8u : OOR, 0u, 0.0);
  // nothing outstanding when the loop starts (vmcnt 0): the compiler's counts at
  // the loop head are then those of the loop's own loads, FD stages deep
  __builtin_amdgcn_s_waitcnt(0x0F70);
  const int ul = lane < NU ? lane : 0;
  double xr = 0.0;
  for (int k0 = 0; k0 < T; k0 += FD) {
#pragma unroll
    for (int d = 0; d < FD; ++d) {
      const int k = k0 + d;
      // the sweep's end leaves the function: a path that left only the unrolled
      // body would reach the loop head with other loads outstanding, and the
      // compiler's wait counts there would drain the prefetch every FD stages
      if (k >= T) return;
      const L<double>* gx = q.gfb + (k * NU + ul) * NX;
      double us = q.gff[k * NU + ul];
      double xn = 0.0;
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        const double xj = lane_read(xr, j);
        us += gx[j] * xj;
        xn += ar[d][j] * xj;
      }
      bdu2.st(lane < NU ? (uint32_t)(k * NU + lane) * 8u : OOR, 0u, us);
#pragma unroll
      for (int u = 0; u < NU; ++u) xn += br[d][u] * lane_read(us, u);
      bdx2.st(lane < NX ? (uint32_t)((k + 1) * NX + lane) * 8u : OOR, 0u, xn);
      xr = xn;
      row_load(ar[d], br[d], k + FD);
    }
  }
}

// Cones are taken CB per lane at a time: the loads of a batch (metadata, then
// gradient rows and states) are issued before its results are stored, so that
// the batch's dependent load chains overlap.
constexpr int CB = 4;

// Set CA_ACT from the iterate (du, dx); returns the number of flags that changed.
// The (du, p) block's cone scans and reductions are shared by the workgroup's
// waves (every wave calls them; red: block-reduction slots).
template <int NX, int NU, typename F>
__device__ int set_active(const Inst<NX, NU, F>& I, const double* dx, const double* du, double* red, int W) {
  int changed = 0;
  const int nt = (int)blockDim.x;
  for (int c0 = (int)threadIdx.x; c0 < I.ng; c0 += CB * nt) {
    double f[CB], old[CB];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int c = c0 + i * nt;
      f[i] = old[i] = 0.0;
      if (c < I.ng) {
        const double a = I.C(CA_BETA, c) + cons_lin<NX, NU, F>(I, c, dx, du);
        f[i] = a > 0.0 ? 1.0 : 0.0;
        old[i] = I.C(CA_ACT, c);
      }
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int c = c0 + i * nt;
      if (c < I.ng) {
        if (f[i] != old[i]) ++changed;
        I.C(CA_ACT, c) = f[i];
      }
    }
  }
  double v[1] = {(double)changed};
  block_sum<1>(red, v, W);   // its barriers also publish CA_ACT to the workgroup
  return (int)v[0];
}

// Exact line search along (du2 - du, dx2 - dx) for the squared-hinge objective.
// Each cone's (a, e) (the constraint's value at the iterate and its change along
// the direction) is kept in the LDS of the Riccati gains (idle until the next
// sweep) when 2 n_g doubles fit there, else in its per-cone columns; the
// piecewise-linear derivative is then evaluated from there at every trial step.
template <int NX, int NU, typename F>
__device__ double line_search(const Inst<NX, NU, F>& I, const QPScratch<NX, NU>& q, double rho, double mu, int W) {
  const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
  const int T = I.T;
  double dHd = 0.0, gd = 0.0;
  for (int idx = tid; idx < T * NU; idx += nt) {
    const int k = idx / NU, u = idx - k * NU;
    double hd = 0.0, hg = 0.0;
#pragma unroll
    for (int w = 0; w < NU; ++w) {
      const double dw = I.du2[k * NU + w] - I.du[k * NU + w];
      hd += I.Ru[u * NU + w] * dw;
      hg += I.Ru[u * NU + w] * (I.uhat[k * NU + w] + I.du[k * NU + w]);
    }
    const double du_ = I.du2[idx] - I.du[idx];
    dHd += 2.0 * hd * du_;
    gd += 2.0 * hg * du_;
  }
  for (int idx = tid; idx < T * NX; idx += nt) {
    const int t = idx / NX + 1, i = idx - (t - 1) * NX;
    double hd = 0.0, hg = 0.0;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double dj = I.dx2[t * NX + j] - I.dx[t * NX + j];
      hd += I.Q[i * NX + j] * dj;
      hg += I.Q[i * NX + j] * (I.xhat[t * NX + j] - I.xg[j] + I.dx[t * NX + j]);
    }
    const double di = I.dx2[t * NX + i] - I.dx[t * NX + i];
    dHd += (2.0 * hd + mu * di) * di;
    gd += (2.0 * hg + mu * I.dx[t * NX + i]) * di;
  }
  const bool in_lds = 2 * I.ng <= T * NU * NX;
  L<double>* lae = q.gfb;   // [2c]: a, [2c + 1]: e
  for (int c0 = tid; c0 < I.ng; c0 += CB * nt) {
    double av[CB], ev[CB];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int c = c0 + i * nt;
      av[i] = ev[i] = 0.0;
      if (c < I.ng) {
        const double a0 = cons_lin<NX, NU, F>(I, c, I.dx, I.du);
        const double a1 = cons_lin<NX, NU, F>(I, c, I.dx2, I.du2);
        av[i] = I.C(CA_BETA, c) + a0;
        ev[i] = a1 - a0;
      }
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int c = c0 + i * nt;
      if (c >= I.ng) continue;
      if (in_lds) {
        lae[2 * c] = av[i];
        lae[2 * c + 1] = ev[i];
      } else {
        I.C(CA_LA, c) = av[i];
        I.C(CA_LE, c) = ev[i];
      }
    }
  }
  {
    double v[2] = {dHd, gd};
    block_sum<2>(q.red, v, W);   // its barriers also publish (a, e)
    dHd = v[0];
    gd = v[1];
  }
  if (dHd <= 0.0) return 0.0;
  auto deriv = [&](double s, double& slope) {
    double f = 0.0, sl = 0.0;
    for (int c = tid; c < I.ng; c += nt) {
      double a, e;
      if (in_lds) {
        a = lae[2 * c];
        e = lae[2 * c + 1];
      } else {
        a = I.C(CA_LA, c);
        e = I.C(CA_LE, c);
      }
      const double z = a + s * e;
      if (z > 0.0) {
        f += e * z;
        sl += e * e;
      }
    }
    double v[2] = {f, sl};
    block_sum<2>(q.red, v, W);
    f = v[0];
    sl = v[1];
    slope = dHd + rho * sl;
    return s * dHd + gd + rho * f;
  };
  double sl0;
  double lo = 0.0, flo = deriv(0.0, sl0);
  if (flo >= 0.0) return 0.0;
  double hi = 1.0, slh;
  double fhi = deriv(hi, slh);
  int guard = 0;
  while (fhi < 0.0 && guard < 60) {
    lo = hi;
    flo = fhi;
    sl0 = slh;
    hi *= 2.0;
    fhi = deriv(hi, slh);
    ++guard;
  }
  if (fhi <= 0.0) return hi;
  double s = lo;
  for (int it = 0; it < 100; ++it) {
    double cand = lo - flo / sl0;          // root of the linear piece to the right of lo
    if (!(cand > lo && cand < hi)) cand = 0.5 * (lo + hi);
    double slc;
    const double fc = deriv(cand, slc);
    s = cand;
    if (fc == 0.0) break;
    if (fc < 0.0) {
      lo = cand;
      flo = fc;
      sl0 = slc;
    } else {
      hi = cand;
    }
    if (hi - lo <= 1e-15 * hi) {
      s = hi;
      break;
    }
    // the piece at lo reaches exactly zero inside (lo, hi): Newton lands on the root next
  }
  return s;
}

// Semismooth Newton at fixed mu from the current iterate (du, dx).  Every wave
// of the workgroup runs it: the Riccati sweep on wave 0, the cone scans, the
// line search and the iterate updates on all waves, with every decision taken
// from block reductions (so block-uniform).
template <int NX, int NU, typename F>
__device__ int ssn(const Inst<NX, NU, F>& I, QPScratch<NX, NU>& q, double rho, double mu, int W) {
  const int T = I.T;
  const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
  set_active<NX, NU, F>(I, I.dx, I.du, q.red, W);
  int solves = 0;
  for (int it = 0; it < 60; ++it) {
    if (wave_id() == 0) riccati<NX, NU, F>(I, q, rho, mu);
    __syncthreads();   // the candidate (du2, dx2) and the gains to every wave
    ++solves;
    // does the candidate keep the active set?
    int changed = 0;
    for (int c0 = tid; c0 < I.ng; c0 += CB * nt) {
#pragma unroll
      for (int i = 0; i < CB; ++i) {
        const int c = c0 + i * nt;
        if (c < I.ng) {
          const double a = I.C(CA_BETA, c) + cons_lin<NX, NU, F>(I, c, I.dx2, I.du2);
          if ((a > 0.0 ? 1.0 : 0.0) != I.C(CA_ACT, c)) ++changed;
        }
      }
    }
    {
      double v[1] = {(double)changed};
      block_sum<1>(q.red, v, W);
      changed = (int)v[0];
    }
    if (changed == 0) {
      for (int i = tid; i < T * NU; i += nt) I.du[i] = I.du2[i];
      for (int i = tid; i < (T + 1) * NX; i += nt) I.dx[i] = I.dx2[i];
      __syncthreads();
      break;
    }
    const double s = line_search<NX, NU, F>(I, q, rho, mu, W);
    double step[1] = {0.0};
    for (int i = tid; i < T * NU; i += nt) {
      const double d = s * (I.du2[i] - I.du[i]);
      step[0] = fmax(step[0], fabs(d));
      I.du[i] += d;
    }
    for (int i = tid; i < (T + 1) * NX; i += nt) I.dx[i] += s * (I.dx2[i] - I.dx[i]);
    block_max<1>(q.red, step, W);   // its barriers also publish (du, dx)
    set_active<NX, NU, F>(I, I.dx, I.du, q.red, W);
    if (step[0] == 0.0) break;
  }
  return solves;
}

template <int NX, int NU, typename F>
__device__ double state_norm(const Inst<NX, NU, F>& I) {
  double s = 0.0;
  for (int i = lane_id(); i < (I.T + 1) * NX; i += NRTO_WAVE) s += I.dx[i] * I.dx[i];
  return sqrt(wave_sum(s));
}

// ||dx|| over the workgroup's waves (block-uniform).
template <int NX, int NU, typename F>
__device__ double state_norm_block(const Inst<NX, NU, F>& I, double* red, int W) {
  double v[1] = {0.0};
  for (int i = (int)threadIdx.x; i < (I.T + 1) * NX; i += (int)blockDim.x) v[0] += I.dx[i] * I.dx[i];
  block_sum<1>(red, v, W);
  return sqrt(v[0]);
}

// Full (du, p) block: returns Riccati solves used.  Requires CA_BETA = g0 + c.
template <int NX, int NU, typename F>
__device__ void rollout_dx(const Inst<NX, NU, F>& I) {
  const int lane = lane_id();
  if (lane < NX) I.dx[lane] = 0.0;
  wave_sync();
  for (int k = 0; k < I.T; ++k) {
    if (lane < NX) {
      const double* A = I.A + (int64_t)k * NX * NX;
      const double* B = I.B + (int64_t)k * NX * NU;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < NX; ++j) s += A[lane * NX + j] * I.dx[k * NX + j];
#pragma unroll
      for (int u = 0; u < NU; ++u) s += B[lane * NU + u] * I.du[k * NU + u];
      I.dx[(k + 1) * NX + lane] = s;
    }
    wave_sync();
  }
}

template <int NX, int NU, typename F>
__device__ __noinline__ int qp_block(const Inst<NX, NU, F> Iarg, QPScratch<NX, NU> qarg, double rho) {
  // compiled out of line with its instance view and LDS carve-up by value; the
  // pointers carry their address spaces and are made wave-uniform (scalar
  // registers) on entry
  const Inst<NX, NU, F> I = uniform_inst(Iarg);
  QPScratch<NX, NU> q = qp_carve<NX, NU>(uni(qarg.V), uni(qarg.gfb), uni(qarg.gff));
  // Trust-region multiplier: mu = 0 if psi(0) = ||F_u du(0)|| <= r, else the
  // root of phi(mu) = 1/r - 1/psi(mu), which increases with mu and is close to
  // linear in it (exactly so when F_u'F_u acts on one eigen-direction of the
  // Hessian).  Safeguarded secant on phi, started from the last multiplier of
  // this instance: a bracket lo < mu* < hi (psi(lo) > r > psi(hi)) is kept once
  // found, steps leaving it become regula falsi / bisection steps, and while no
  // upper end is known the multiplier grows by at most 16x per step.
  const double r = I.r_trust;
  const double tol = 1e-13 * r;
  const int W = (int)(blockDim.x / NRTO_WAVE);
  int solves = 0;
  if (wave_id() == 0) {
    L<int>* tl = (L<int>*)q.tl;
    for (int i = lane_id(); i < 2 * I.T + 3; i += NRTO_WAVE) tl[i] = I.tls[i];   // tls then tlc
    wave_sync();
    rollout_dx<NX, NU, F>(I);
  }
  __syncthreads();
  auto eval = [&](double m) {
    solves += ssn<NX, NU, F>(I, q, rho, m, W);
    return state_norm_block<NX, NU, F>(I, q.red, W);
  };
  // start: when the last block ended with an inactive trust region (mu = 0, also
  // at a cold start), mu = 0 first -- a single evaluation whenever the region
  // stays inactive -- and, if psi(0) > r, the last positive multiplier of this
  // instance (kept across solves) or 1; otherwise the current multiplier, then
  // mu = 0 when psi(start) < r
  double lo = 0.0, flo = 0.0, hi = -1.0, fhi = 0.0;   // hi < 0: no upper end yet
  bool have_lo = false;
  double m0 = 0.0, f0 = 0.0, m1, f1;
  bool have_prev = false;
  bool done;
  double mu, psi;
  if (!(*I.mu > 0.0)) {
    mu = 0.0;
    psi = eval(0.0);
    m1 = 0.0;
    f1 = 1.0 / r - 1.0 / psi;
    done = psi <= r + tol;
    if (!done) {
      lo = 0.0;
      flo = f1;
      have_lo = true;
      m0 = m1;
      f0 = f1;
      have_prev = true;
      mu = (I.iscr[ISCR_MUHINT] > 0.0) ? I.iscr[ISCR_MUHINT] : 1.0;
      psi = eval(mu);
      m1 = mu;
      f1 = 1.0 / r - 1.0 / psi;
      done = fabs(psi - r) <= tol;
      if (!done && psi < r) {
        hi = mu;
        fhi = f1;
      }
    }
  } else {
    mu = *I.mu;
    psi = eval(mu);
    m1 = mu;
    f1 = 1.0 / r - 1.0 / psi;
    done = fabs(psi - r) <= tol;
    if (!done && psi < r) {
      // the root lies below the last multiplier, possibly at mu = 0
      hi = mu;
      fhi = f1;
      m0 = m1;
      f0 = f1;
      have_prev = true;
      psi = eval(0.0);
      m1 = 0.0;
      f1 = 1.0 / r - 1.0 / psi;
      mu = 0.0;
      done = psi <= r + tol;
    }
  }
  if (!done) {
    if (psi > r) {
      lo = m1;
      flo = f1;
      have_lo = true;
    }
    for (int it = 0; it < 80; ++it) {
      double m2;
      if (have_prev && f1 != f0) m2 = m1 - f1 * (m1 - m0) / (f1 - f0);
      else m2 = (m1 > 0.0) ? m1 * psi / r : 1.0;   // phi linear in mu with zero offset
      if (hi > 0.0) {
        if (!(m2 > lo && m2 < hi)) m2 = lo - flo * (hi - lo) / (fhi - flo);
        if (!(m2 > lo && m2 < hi)) m2 = 0.5 * (lo + hi);
      } else {
        const double base = fmax(lo, 1.0);
        if (!(m2 > lo)) m2 = 4.0 * base;
        if (m2 > 16.0 * base) m2 = 16.0 * base;
      }
      m0 = m1;
      f0 = f1;
      have_prev = true;
      m1 = m2;
      psi = eval(m1);
      f1 = 1.0 / r - 1.0 / psi;
      mu = m1;
      if (fabs(psi - r) <= tol) break;
      if (psi > r) {
        lo = m1;
        flo = f1;
        have_lo = true;
      } else {
        hi = m1;
        fhi = f1;
      }
      if (hi > 0.0 && hi - lo <= 1e-15 * hi) break;
    }
  }
  (void)have_lo;
  if (threadIdx.x == 0) {
    *I.mu = mu;
    I.iscr[ISCR_PSI] = psi;
    if (mu > 0.0) I.iscr[ISCR_MUHINT] = mu;
  }
  __syncthreads();
  return solves;
}

// ----------------------------------------------------------------------------
// KKT check entry pass: per cone ||eta||^2, ||zeta||^2, zeta.eta, and the
// adjoint sum_j A_hat_j' zeta_j into acc (K read from kk).  Static schedule over
// the wave tasks; a long cone is one wave's (its block vectors staged in the
// wave's LDS slice, its entries loaded 256 at a time), packed short cones take
// one entry per lane with per-cone sums formed by a segmented suffix sum over
// the lanes (fixed order).  Compiled on its own (like the DR pass), with the
// instance view by value and made wave-uniform.
template <int NX, int NU, typename F, int METHOD, typename AccP, typename KP>
__device__ __noinline__ void kkt_entry_pass(const Inst<NX, NU, F> Iarg, AccP acc, KP kk, L<F>* bl_all, double sig,
                                            double rho_fa, int pending_i, int w0) {
  if ((int)wave_id() < w0) return;   // waves below w0 take no task
  const Inst<NX, NU, F> I = uniform_inst(Iarg);
  const int T = I.T;
  const double r = I.r;
  const bool pending = pending_i != 0;
  const int W = (int)(blockDim.x / NRTO_WAVE);
  const int lane = lane_id();
  F* bl = bl_all + wave_id() * (T + 1) * NU;
  // eta and zeta of entry e of a cone (s~ and b_hat of the entry already
  // loaded), block k, component x, block vector bv
  auto eta_zeta = [&](int64_t e, double st_e, double bh_e, int k, int x, const F* bv, double& eta, double& z) {
    double f = 0.0;
    if (k < T) {
#pragma unroll
      for (int u = 0; u < NU; ++u) f += (double)bv[u] * kk[(k * NU + u) * NX + x];
    }
    eta = r * f + bh_e;
    if (METHOD == NRTO_DR) {
      z = sig * (st_e - eta);
    } else {
      double lv = st_e;
      if (pending) lv += eta - (double)I.nuv[e];
      z = -rho_fa * lv;
    }
  };
  auto adjoint = [&](int k, int x, const F* bv, double z) {
    if (k >= T) return;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const double cz = r * (double)bv[u] * z;
      if (cz != 0.0) atomicAdd(&acc[(k * NU + u) * NX + x], cz);
    }
  };
  for (int t = uni((int)wave_id()) - w0; t < I.ntask; t += W - w0) {
    const WaveTask tk = I.tasks[t];
    if (tk.ncone == 1 && tk.len > NRTO_WAVE) {
      const int c = tk.cone, len = tk.len, k0 = tk.k0;
      const G<F>* bvp = I.bvec + (int64_t)tk.boff * NU;
      const int nbv = ((len - 1) / NX) * NU;
      BlockStage<F> bs;
      bs.load(bvp, nbv, 0);
      bs.store(bl, nbv, 0);
      bs.rest(bvp, nbv, bl);
      wave_sync();
      double n2 = 0.0, z2 = 0.0, ze = 0.0;
      constexpr int E = 4;
      for (int base = 0; base < len; base += E * NRTO_WAVE) {
        // the group's loads first, so that they are in flight together
        double stv[E], bhv[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int le = base + lane + i * NRTO_WAVE;
          const bool in = le >= 1 && le < len;
          stv[i] = in ? (double)I.st[tk.ebeg + le] : 0.0;
          bhv[i] = in ? (double)I.bhat[tk.ebeg + le] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int le = base + lane + i * NRTO_WAVE;
          if (le >= 1 && le < len) {
            const int q = le - 1, blk = q / NX, x = q - blk * NX, k = k0 + blk;
            double eta, z;
            eta_zeta(tk.ebeg + le, stv[i], bhv[i], k, x, bl + blk * NU, eta, z);
            n2 += eta * eta;
            z2 += z * z;
            ze += z * eta;
            adjoint(k, x, bl + blk * NU, z);
          }
        }
      }
      n2 = wave_sum(n2);
      z2 = wave_sum(z2);
      ze = wave_sum(ze);
      if (lane == 0) {
        I.C(CA_N, c) = sqrt(n2);
        I.C(CA_ZZ, c) = z2;
        I.C(CA_ZE, c) = ze;
      }
      wave_sync();   // the slice is reused by the wave's next cone
    } else {
      const uint64_t mask = I.tmask[t];
      const int l = lane;
      const uint64_t pre = mask & ((l == 63) ? ~0ull : ((2ull << l) - 1ull));
      const uint64_t above = mask & ~((l == 63) ? ~0ull : ((2ull << l) - 1ull));
      const int cl = __popcll(pre) - 1;
      const int cs = 63 - __clzll(pre);
      const int ce = above ? __ffsll((unsigned long long)above) - 1 : tk.len;   // end of this lane's cone
      const int le = l - cs;
      const int c = tk.cone + cl;
      double n2 = 0.0, z2 = 0.0, ze = 0.0;
      if (l < tk.len && le >= 1) {
        // block time and block vector of the lane's entry from the lane table
        // (k = -1: a block without gain)
        const LaneBlock lb = I.lblock[(int64_t)(t - I.nlong) * NRTO_WAVE + l];
        const int x = (le - 1) % NX;
        const int k = lb.k >= 0 ? lb.k : T;
        const F* bv = I.bvec + (int64_t)(lb.k >= 0 ? lb.b : 0) * NU;
        double eta, z;
        eta_zeta(tk.ebeg + l, (double)I.st[tk.ebeg + l], (double)I.bhat[tk.ebeg + l], k, x, bv, eta, z);
        n2 = eta * eta;
        z2 = z * z;
        ze = z * eta;
        adjoint(k, x, bv, z);
      }
      // segmented suffix sums: lane l ends with the sum over [l, ce)
#pragma unroll
      for (int off = 1; off < NRTO_WAVE; off <<= 1) {
        const double a = __shfl_down(n2, off, NRTO_WAVE);
        const double b = __shfl_down(z2, off, NRTO_WAVE);
        const double d = __shfl_down(ze, off, NRTO_WAVE);
        if (l + off < ce) {
          n2 += a;
          z2 += b;
          ze += d;
        }
      }
      if (l < tk.len && le == 0) {
        I.C(CA_N, c) = sqrt(n2);
        I.C(CA_ZZ, c) = z2;
        I.C(CA_ZE, c) = ze;
      }
    }
  }
}

// T1 of the KKT residual: the input-stationarity term, from three costate
// recursions run backward over the horizon on one wave (lanes 0..NX-1 the cost
// costate, NX..2NX-1 the constraint-multiplier costate, 2NX..3NX-1 the
// trust-region costate).  The costates stay in registers and are read across
// lanes; the cone loops issue their loads four cones at a time.  Every lane
// returns the value.
template <int NX, int NU, typename F>
__device__ __noinline__ double kkt_t1(const Inst<NX, NU, F> Iarg) {
  static_assert(3 * NX <= NRTO_WAVE, "three costates in one wave");
  const Inst<NX, NU, F> I = uniform_inst(Iarg);
  const int T = I.T;
  const int lane = lane_id();
  const int which = lane / NX, i = lane - which * NX;
  const double mu = *I.mu;
  double qrow[NX], xg[NX], ru[NU];
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    qrow[j] = I.Q[i * NX + j];
    xg[j] = I.xg[j];
  }
#pragma unroll
  for (int w = 0; w < NU; ++w) ru[w] = lane < NU ? I.Ru[lane * NU + w] : 0.0;
  double lam = 0.0;
  double g1m = 0.0, g2m = 0.0, g3m = 0.0, gsm = 0.0;
  for (int t = T; t >= 1; --t) {
    const int k = t - 1;
    // the stage's loads first, so that they are in flight together: lane i's
    // column of A_k, row lane of B_k' (lanes below NU) and u_k + du_k
    double av[NX], bv[NX], ud[NU];
    {
      const double* A = I.A + (int64_t)k * NX * NX;
      const double* B = I.B + (int64_t)k * NX * NU;
      const int bl = lane < NU ? lane : 0;
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        av[j] = A[j * NX + i];
        bv[j] = B[j * NU + bl];
      }
#pragma unroll
      for (int w = 0; w < NU; ++w) ud[w] = I.uhat[k * NU + w] + I.du[k * NU + w];
    }
    // stage terms of time t
    double add = 0.0;
    if (which == 0) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < NX; ++j) s += qrow[j] * (I.xhat[t * NX + j] - xg[j] + I.dx[t * NX + j]);
      add = 2.0 * s;
    } else if (which == 1) {
      const int c1 = I.tls[t + 1];
      for (int c = I.tls[t]; c < c1; c += 4) {
        double pv[4], wv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const bool in = c + b < c1;
          pv[b] = in ? I.C(CA_PI, c + b) : 0.0;
          wv[b] = in ? I.W[(int64_t)(c + b) * NX + i] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (c + b < c1) add += pv[b] * wv[b];
      }
    } else if (which == 2) {
      add = mu * I.dx[t * NX + i];
    }
    lam += add;
    // gradients at step k from lambda_{k+1}, and lambda_k = A_k' lambda_{k+1}
    double g1 = 0.0, g2 = 0.0, g3 = 0.0;
#pragma unroll
    for (int w = 0; w < NU; ++w) g1 += ru[w] * ud[w];
    g1 *= 2.0;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double l0 = lane_read(lam, j), l1 = lane_read(lam, NX + j), l2 = lane_read(lam, 2 * NX + j);
      g1 += bv[j] * l0;
      g2 += bv[j] * l1;
      g3 += bv[j] * l2;
      s += av[j] * (which == 0 ? l0 : (which == 1 ? l1 : l2));
    }
    if (lane < NU) {
      const int c1 = I.tlc[k + 1];
      for (int c = I.tlc[k]; c < c1; c += 4) {
        double pv[4];
        int ci[4], cs[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const bool in = c + b < c1;
          const int32_t* m = I.cm + (int64_t)(in ? c + b : c) * CM_N;
          ci[b] = in ? m[CM_CIDX] : -1;
          cs[b] = m[CM_CSIGN];
          pv[b] = in ? I.C(CA_PI, c + b) : 0.0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (ci[b] == lane) g2 += pv[b] * (double)cs[b];
      }
      g1m = fmax(g1m, fabs(g1));
      g2m = fmax(g2m, fabs(g2));
      g3m = fmax(g3m, fabs(g3));
      gsm = fmax(gsm, fabs(g1 + g2 + g3));
    }
    lam = which < 3 ? s : 0.0;
  }
  g1m = wave_max(g1m);
  g2m = wave_max(g2m);
  g3m = wave_max(g3m);
  gsm = wave_max(gsm);
  return gsm / (1.0 + fmax(g1m, fmax(g2m, g3m)));
}

// FP64 KKT residual (see the oracle's definition).  Uses K (double), the
// multipliers CA_PI, mu, and zeta from the method state.
template <int NX, int NU, typename F, int METHOD>
__device__ double kkt_residual(const Inst<NX, NU, F>& I, Smem<F>& S, const SolveOpts& o, double sig, bool pending,
                               int W) {
  const int T = I.T;
  // accumulator of sum_j A_hat_j' zeta_j, [(k*NU + u)*NX + x].  In the FP64
  // form it takes the LDS of the adjoint accumulator Racc, whose contents (the
  // next K-solve's input) are saved to global scratch meanwhile and restored at
  // the end, and K is read from the LDS of the gain copy Kf (idle from the
  // (du, p) block to the next K-solve); else the accumulator is global scratch
  // and K is read from global memory.
  // With more than one wave, wave 0 runs the T1 recursion (which reads none of
  // what the entry pass writes) while the other waves take the entry tasks.
  const int w0 = W > 1 ? 1 : 0;
  auto t1_wave0 = [&]() {
    const double v = kkt_t1<NX, NU, F>(I);
    if (lane_id() == 0) S.red[64] = v;
  };
  if constexpr (sizeof(F) == 8) {
    L<double>* acc = (L<double>*)S.Racc;
    L<double>* kl = (L<double>*)S.Kf;
    for (int i = threadIdx.x; i < T * NU * NX; i += blockDim.x) {
      I.kscr[i] = acc[i];
      acc[i] = 0.0;
      kl[i] = I.K[i];
    }
    __syncthreads();
    if (w0 && wave_id() == 0) t1_wave0();
    else kkt_entry_pass<NX, NU, F, METHOD>(I, acc, (const L<double>*)kl, S.bl, sig, o.rho, pending ? 1 : 0, w0);
  } else {
    for (int i = threadIdx.x; i < T * NU * NX; i += blockDim.x) I.kscr[i] = 0.0;
    __syncthreads();
    if (w0 && wave_id() == 0) t1_wave0();
    else kkt_entry_pass<NX, NU, F, METHOD>(I, I.kscr, (const G<double>*)I.K, S.bl, sig, o.rho, pending ? 1 : 0, w0);
  }
  if (!w0) t1_wave0();   // a single wave: after its entry tasks
  __syncthreads();
  // per-cone terms
  double mx[4] = {0.0, 0.0, 0.0, 0.0};   // T3 num, T5 num, T6 num, T7 num
  double nm[4] = {0.0, 0.0, 0.0, 0.0};   // max|g0|, max|b'du|, max n, max pi
  double nm2[4] = {0.0, 0.0, 0.0, 0.0};  // max|e|, max pi*n, T8 num, max|p|,|pt|
  for (int c = threadIdx.x; c < I.ng; c += blockDim.x) {
    const double g0 = I.C(CA_G0, c);
    const double bdu = cons_lin<NX, NU, F>(I, c, I.dx, I.du);
    const double e = g0 + bdu;
    const double n = I.C(CA_N, c);
    const double pi = I.C(CA_PI, c);
    const double zz = sqrt(I.C(CA_ZZ, c));
    const double ze = I.C(CA_ZE, c);
    const double p = I.C(CA_P, c), pt = I.C(CA_PT, c);
    I.C(CA_E, c) = e;
    const double viol = e + n;
    mx[0] = fmax(mx[0], viol);
    mx[1] = fmax(mx[1], fabs(p - pt));
    mx[2] = fmax(mx[2], fabs(fmin(pi, -viol)));
    mx[3] = fmax(mx[3], fmax(-pi, zz - pi));
    nm[0] = fmax(nm[0], fabs(g0));
    nm[1] = fmax(nm[1], fabs(bdu));
    nm[2] = fmax(nm[2], n);
    nm[3] = fmax(nm[3], pi);
    nm2[0] = fmax(nm2[0], fabs(e));
    nm2[1] = fmax(nm2[1], pi * n);
    nm2[2] = fmax(nm2[2], fabs(pi * n + ze));
    nm2[3] = fmax(nm2[3], fmax(fabs(p), fabs(pt)));
  }
  // T2: Q_v k - sum A_hat' zeta
  double t2[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < T * NU * NX; i += blockDim.x) {
    const int k = i / (NU * NX), rem = i - k * NU * NX, u = rem / NX, x = rem - u * NX;
    double qk = 0.0;
#pragma unroll
    for (int w = 0; w < NU; ++w) qk += I.RK2[u * NU + w] * I.K[(k * NU + w) * NX + x];
    qk *= 2.0;
    double az;
    if constexpr (sizeof(F) == 8) az = ((const L<double>*)S.Racc)[i];
    else az = atomic_load_agent(&I.kscr[i]);
    t2[0] = fmax(t2[0], fabs(qk - az));
    t2[1] = fmax(t2[1], fabs(qk));
    t2[2] = fmax(t2[2], fabs(az));
  }
  block_max<4>(S.red, mx, W);
  block_max<4>(S.red, nm, W);
  block_max<4>(S.red, nm2, W);
  block_max<4>(S.red, t2, W);
  const double t1v = S.red[64];
  const double rt = I.r_trust;
  const double psi = I.iscr[ISCR_PSI];
  const double mu = *I.mu;
  double res = t1v;
  res = fmax(res, t2[0] / (1.0 + fmax(t2[1], t2[2])));
  res = fmax(res, fmax(0.0, mx[0]) / (1.0 + fmax(nm[0], fmax(nm[1], nm[2]))));
  res = fmax(res, fmax(0.0, psi - rt) / (1.0 + rt));
  res = fmax(res, mx[1] / (1.0 + nm2[3]));
  res = fmax(res, mx[2] / (1.0 + fmax(nm[3], fmax(nm2[0], nm[2]))));
  res = fmax(res, fmax(0.0, mx[3]) / (1.0 + nm[3]));
  res = fmax(res, nm2[2] / (1.0 + nm2[1]));
  res = fmax(res, fabs(fmin(mu, rt - psi)) / (1.0 + fmax(mu, rt)));
  __syncthreads();
  if constexpr (sizeof(F) == 8) {   // the next K-solve's adjoint back into Racc
    L<double>* acc = (L<double>*)S.Racc;
    for (int i = threadIdx.x; i < T * NU * NX; i += blockDim.x) acc[i] = I.kscr[i];
    __syncthreads();
  }
  return res;
}

// ----------------------------------------------------------------------------
template <int NX, int NU, typename F>
__device__ void zero_state(const Inst<NX, NU, F>& I) {
  const int T = I.T;
  for (int64_t e = threadIdx.x; e < I.nent; e += blockDim.x) {
    I.st[e] = (F)0;
    I.nuv[e] = (F)0;
  }
  for (int c = threadIdx.x; c < I.ng; c += blockDim.x) {
    I.C(CA_P, c) = 0.0;
    I.C(CA_PT, c) = 0.0;
    I.C(CA_PTT, c) = 0.0;
    I.C(CA_LAM, c) = 0.0;
    I.C(CA_PI, c) = 0.0;
    I.C(CA_ACT, c) = 0.0;
  }
  for (int i = threadIdx.x; i < T * NU * NX; i += blockDim.x) {
    I.K[i] = 0.0;
    I.Kt[i] = 0.0;
  }
  for (int i = threadIdx.x; i < T * NU; i += blockDim.x) I.du[i] = 0.0;
  for (int i = threadIdx.x; i < (T + 1) * NX; i += blockDim.x) I.dx[i] = 0.0;
  if (threadIdx.x == 0) {
    *I.mu = 0.0;
    I.flags[0] = 0;
    I.iscr[ISCR_PSI] = 0.0;
    I.iscr[ISCR_MUHINT] = 0.0;   // a cold solve keeps nothing from earlier solves
  }
  __syncthreads();
}

// Change of the DR scaling sigma_s -> sigma_s / f keeping the cone multiplier
// estimate: s~ <- S + f (s~ - S) with S = (p~, eta(K)) of the last DR iteration,
// and the adjoint accumulator rebuilt from the new s~.
template <int NX, int NU, typename F>
__device__ void rescale_pass(const Inst<NX, NU, F>& I, Smem<F>& S, double f) {
  const int T = I.T;
  const F r = (F)I.r;
  for (int i = threadIdx.x; i < NU * T * NX; i += blockDim.x) S.Racc[i] = (F)0;
  if (threadIdx.x == 0) *S.ctr = 0;
  __syncthreads();
  for (int t = next_task(S.ctr); t < I.ntask; t = next_task(S.ctr)) {
    const WaveTask tk = I.tasks[t];
    for (int c = tk.cone; c < tk.cone + tk.ncone; ++c) {
      const int32_t* m = I.cm + c * CM_N;
      const int e0 = m[CM_EOFF];
      const int len = 1 + m[CM_NBLK] * NX;
      for (int le = lane_id(); le < len; le += NRTO_WAVE) {
        const int64_t e = e0 + le;
        if (le == 0) {
          const double sv = I.C(CA_PT, c);
          I.st[e] = (F)(sv + f * ((double)I.st[e] - sv));
        } else {
          int k, x, b;
          entry_block<NX>(m, le, k, x, b);
          const F bh = I.bhat[e];
          const F sv = r * fwd_gemm<NX, NU, F>(I, S, T, k, x, I.bvec + (int64_t)b * NU) + bh;
          const F sn = (F)((double)sv + f * ((double)I.st[e] - (double)sv));
          I.st[e] = sn;
          adj_gemm<NX, NU, F>(S, T, k, x, I.bvec + (int64_t)b * NU, sn - bh);
        }
      }
    }
  }
  __syncthreads();
}

// Open-loop cold point (DR): every cone at its value for k_v = 0,
// s~_j = (||b_hat_j||, b_hat_j) and p = p~ = p~~ = ||b_hat_j||.
template <int NX, int NU, typename F>
__device__ void margin_pass(const Inst<NX, NU, F>& I, Smem<F>& S) {
  for (int t = next_task(S.ctr); t < I.ntask; t = next_task(S.ctr)) {
    const WaveTask tk = I.tasks[t];
    for (int c = tk.cone; c < tk.cone + tk.ncone; ++c) {
      const int32_t* m = I.cm + c * CM_N;
      const int e0 = m[CM_EOFF];
      const int len = 1 + m[CM_NBLK] * NX;
      double n2 = 0.0;
      for (int le = 1 + lane_id(); le < len; le += NRTO_WAVE) {
        const double b = (double)I.bhat[e0 + le];
        n2 += b * b;
        I.st[e0 + le] = I.bhat[e0 + le];
      }
      const double nrm = sqrt(wave_sum(n2));
      if (lane_id() == 0) {
        I.st[e0] = (F)nrm;
        I.C(CA_P, c) = nrm;
        I.C(CA_PT, c) = nrm;
        I.C(CA_PTT, c) = nrm;
      }
    }
  }
}

// The cold point of a solve: zeros, or the open-loop point when cold_init is set
// (NRTO-DR only).
template <int NX, int NU, typename F, int METHOD>
__device__ void cold_state(const Inst<NX, NU, F>& I, Smem<F>& S, const SolveOpts& o) {
  zero_state<NX, NU, F>(I);
  if (METHOD == NRTO_DR && o.cold_init) {
    if (threadIdx.x == 0) *S.ctr = 0;
    __syncthreads();
    margin_pass<NX, NU, F>(I, S);
    __syncthreads();
  }
  for (int c = threadIdx.x; c < I.ng; c += blockDim.x) I.C(CA_PTP, c) = I.C(CA_PT, c);
  __syncthreads();
}

template <int NX, int NU, typename F, int METHOD>
__device__ void solve_instance(const DevPtrs& g, const SolveOpts& o, int ii, L<char>* smem) {
  // a continuation launch of a chunked solve only runs instances that reached
  // the previous launch's iteration limit (block-uniform: one report per block)
  nrto_solve_report prev;
  if (o.cont) {
    prev = g.rep[ii];
    if (prev.status != NRTO_MAXITER) return;
  }
  Inst<NX, NU, F> I = make_inst<NX, NU, F>(g, ii);
  const int W = blockDim.x / NRTO_WAVE;
  Smem<F> S = carve<F>(smem, I.T, NX, NU, W);
  double rho = (o.cont && prev.rho > 0.0) ? prev.rho : o.rho;
  // phase timers (device wall clock ticks, read by thread 0 after block barriers)
  const long long t_start = wall_clock64();
  long long t_dr = 0, t_qp = 0, t_kkt = 0, t_mark = 0;

  if (!o.warm) cold_state<NX, NU, F, METHOD>(I, S, o);
  for (int c = threadIdx.x; c < I.ng; c += blockDim.x) I.C(CA_PTP, c) = I.C(CA_PT, c);
  __syncthreads();
  bool pending = I.flags[0] != 0;
  // current DR scaling: the option's value at a cold start, else the one the last
  // solve of this instance ended with (kept in its report)
  double sig = o.warm ? g.rep[ii].sigma_s : o.sigma_s;
  if (!(sig > 0.0)) sig = o.sigma_s;
  __syncthreads();

  // a1: factor the reduced KKT blocks once
  if (METHOD == NRTO_DR)
    factor_blocks<NX, NU, F>(I, S, sig * I.r * I.r, o.sigma_chi);
  else
    factor_blocks<NX, NU, F>(I, S, rho * I.r * I.r, 0.0);

  load_kf<NX, NU, F>(I, S);
  if (METHOD == NRTO_DR) {
    if (threadIdx.x == 0) *S.ctr = 0;
    __syncthreads();
    r_pass<NX, NU, F>(I, S);
    __syncthreads();
  }

  // a continuation launch counts on from the previous launch of the solve, so
  // that the schedules that depend on the counts (sigma_s balancing every
  // sigma_every DR iterations, the KKT check every check_every ADMM iterations)
  // are those of one launch
  const int l0 = o.cont ? prev.admm_iters : 0;
  int admm = l0, inner = o.cont ? prev.inner_iters : 0, qpn = o.cont ? prev.qp_newton : 0;
  int status = NRTO_MAXITER, sig_updates = o.cont ? prev.sigma_updates : 0, nan_flag = 0;
  double rp_best = 1e300;   // smallest consensus residual so far and its ADMM iteration
  int l_best = l0;
  double kkt = 1e300, rp = 0.0, rd = 0.0;
  const int l_end = l0 + o.max_admm;
  for (int l = l0 + 1; l <= l_end; ++l) {
    admm = l;
    t_mark = wall_clock64();
    if (METHOD == NRTO_DR) {
      // (6a) DR iterations on the {k_v, p~} block, warm-started
      for (int i = 0; i < o.max_inner; ++i) {
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        {
          double kacc[2] = {0.0, 0.0};
          k_solve<NX, NU, F, NRTO_DR>(I, S, o, sig, kacc);
          acc[2] = kacc[0];
          acc[3] = kacc[1];
        }
        if (threadIdx.x == 0) *S.ctr = 0;
        __syncthreads();
        dr_pass<NX, NU, F>(I, S, o, rho, sig, acc);
        block_sum<5>(S.red, acc, W);
        ++inner;
        const double rdr = sqrt(acc[0]);
        if (o.sigma_adapt && inner % o.sigma_every == 0) {
          // balance of the DR scaling (block-uniform: acc comes from block sums)
          const double n_s = fmax(1.0, sqrt(acc[4]));
          const double n_k = fmax(1.0, sqrt(acc[3]));
          const double r_prim = rdr / o.alpha;
          const double r_dual = sqrt(acc[2]);
          if (r_prim > 1e-9 * n_s && r_dual > 1e-9 * n_k) {
            const double ratio = sqrt((r_prim / n_s) / (r_dual / n_k));
            if (ratio > o.sigma_thr || ratio < 1.0 / o.sigma_thr) {
              const double nsig = fmin(fmax(sig * ratio, o.sigma_min), o.sigma_max);
              if (nsig != sig) {
                rescale_pass<NX, NU, F>(I, S, sig / nsig);
                sig = nsig;
                ++sig_updates;
                factor_blocks<NX, NU, F>(I, S, sig * I.r * I.r, o.sigma_chi);
              }
            }
          }
        }
        if (rdr <= o.eps_dr_abs + o.eps_dr_rel * fmax(1.0, sqrt(acc[1]))) break;
      }
      // p~ of the last chi is in CA_PT, k_v of the last chi in K
      for (int c = threadIdx.x; c < I.ng; c += blockDim.x)
        I.C(CA_BETA, c) = I.C(CA_G0, c) + I.C(CA_PT, c) - I.C(CA_LAM, c) / rho;
    } else {
      if (threadIdx.x == 0) *S.ctr = 0;
      __syncthreads();
      double acc[2] = {0.0, 0.0};
      fa_pass<NX, NU, F>(I, S, o, pending, acc);
      pending = true;
      block_sum<2>(S.red, acc, W);
      rd = rho * sqrt(acc[1]);
      for (int c = threadIdx.x; c < I.ng; c += blockDim.x)
        I.C(CA_BETA, c) = I.C(CA_G0, c) + I.C(CA_PT, c) - I.C(CA_LAM, c);
    }
    __syncthreads();
    {
      const long long now = wall_clock64();
      t_dr += now - t_mark;
      t_mark = now;
    }
    // (du, p) block: Riccati sweeps on wave 0, cone scans on every wave
    {
      QPScratch<NX, NU> q = qp_carve<NX, NU>(S.qp, S.gfb, S.gff);
      qpn += qp_block<NX, NU, F>(I, q, rho);
    }
    {
      const long long now = wall_clock64();
      t_qp += now - t_mark;
      t_mark = now;
    }
    // p, pi from the (du, p) solution; then the FullADMM k_v step; dual updates
    double acc2[3] = {0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < I.ng; c += blockDim.x) {
      const double a = cons_lin<NX, NU, F>(I, c, I.dx, I.du);
      const double g0 = I.C(CA_G0, c);
      const double cc = I.C(CA_BETA, c) - g0;
      const double p = fmin(cc, -(g0 + a));
      const double pi = rho * fmax(0.0, g0 + a + cc);
      const double pt = I.C(CA_PT, c);
      I.C(CA_P, c) = p;
      I.C(CA_PI, c) = pi;
      if (METHOD == NRTO_DR) {
        const double lam_old = I.C(CA_LAM, c);
        I.C(CA_LAM, c) = lam_old + rho * (p - pt);
        const double dpt = pt - I.C(CA_PTP, c);
        acc2[1] += dpt * dpt;
        I.C(CA_PTP, c) = pt;
      } else {
        I.C(CA_LAM, c) = I.C(CA_LAM, c) + (p - pt);
      }
      acc2[0] += (p - pt) * (p - pt);
      acc2[2] += pt * pt;
    }
    if (METHOD == NRTO_FULLADMM) {
      double kacc[2] = {0.0, 0.0};
      k_solve<NX, NU, F, NRTO_FULLADMM>(I, S, o, sig, kacc);
    }
    block_sum<3>(S.red, acc2, W);
    rp = sqrt(acc2[0]);
    if (isnan(rp)) {   // NaN inputs propagate; stop and flag (block-uniform)
      nan_flag = 1;
      break;
    }
    if (METHOD == NRTO_DR) rd = rho * sqrt(acc2[1]);
    if (o.eps_kkt > 0.0 && (l % o.check_every == 0 || l == l_end)) {
      kkt = kkt_residual<NX, NU, F, METHOD>(I, S, o, sig, pending, W);
      t_kkt += wall_clock64() - t_mark;
      if (kkt <= o.eps_kkt) {
        status = NRTO_OK;
        break;
      }
    }
    // stagnating consensus residual: no 1% decrease within infeas_window ADMM iterations
    if (METHOD == NRTO_DR && o.infeas_window > 0) {
      if (rp < 0.99 * rp_best) {
        rp_best = rp;
        l_best = l;
      }
      if (l - l_best >= o.infeas_window && rp > 1e-3 * (1.0 + sqrt(acc2[2]))) {
        status = NRTO_INFEASIBLE;
        break;
      }
    }
    // residual balancing of the penalty (block-uniform: rp, rd come from block sums)
    if (METHOD == NRTO_DR && o.rho_adapt) {
      if (rp > o.rho_mu * rd) rho = fmin(o.rho_max, rho * o.rho_tau);
      else if (rd > o.rho_mu * rp) rho = fmax(o.rho_min, rho / o.rho_tau);
    }
  }
  if (METHOD == NRTO_FULLADMM && pending) {
    if (threadIdx.x == 0) *S.ctr = 0;
    __syncthreads();
    fa_commit<NX, NU, F>(I, S);
    pending = false;
    __syncthreads();
  }
  if (!(o.eps_kkt > 0.0)) kkt = kkt_residual<NX, NU, F, METHOD>(I, S, o, sig, false, W);
  if (threadIdx.x == 0) {
    I.flags[0] = pending ? 1 : 0;
    nrto_solve_report rep;
    rep.status = status;
    rep.admm_iters = admm;
    rep.inner_iters = inner;
    rep.qp_newton = qpn;
    rep.kkt = kkt;
    rep.r_p = rp;
    rep.r_d = rd;
    rep.mu = *I.mu;
    rep.rho = rho;
    rep.sigma_s = sig;
    rep.sigma_updates = sig_updates;
    rep.nan_flag = (nan_flag || isnan(kkt)) ? 1 : 0;
    // ticks here; the host scales them to microseconds
    rep.t_dr_us = (double)t_dr;
    rep.t_qp_us = (double)t_qp;
    rep.t_kkt_us = (double)t_kkt;
    rep.t_total_us = (double)(wall_clock64() - t_start);
    if (o.cont) {   // times of the whole solve (the counts went on from the previous launch)
      rep.nan_flag = (rep.nan_flag || prev.nan_flag) ? 1 : 0;
      rep.t_dr_us += prev.t_dr_us;
      rep.t_qp_us += prev.t_qp_us;
      rep.t_kkt_us += prev.t_kkt_us;
      rep.t_total_us += prev.t_total_us;
    }
    g.rep[ii] = rep;
  }
}

// ----------------------------------------------------------------------------
// Learned warm start for NRTO-DR: set the method state from a prediction
// (du, K, p~, pi) through the DR fixed-point relations with the cold point's
// gains K = K~ = 0: p~ = max(predicted p~_j, ||eta_j||), p = p~~ = p~,
// lambda = -pi, s = (p~, eta), y_j = pi_j (1, -eta_j / ||eta_j||) (zero when
// eta_j = 0), s~ = s + y / sigma_s.  The KKT residual of the warm point is
// compared with that of the cold point; the cold point is kept when the warm one
// is worse.
template <int NX, int NU, typename F>
__device__ void warm_pass(const Inst<NX, NU, F>& I, Smem<F>& S, const SolveOpts& o) {
  const int T = I.T;
  const F r = (F)I.r;
  const double inv_s = 1.0 / o.sigma_s;
  for (int t = next_task(S.ctr); t < I.ntask; t = next_task(S.ctr)) {
    const WaveTask tk = I.tasks[t];
    for (int c = tk.cone; c < tk.cone + tk.ncone; ++c) {
      const int32_t* m = I.cm + c * CM_N;
      const int e0 = m[CM_EOFF];
      const int len = 1 + m[CM_NBLK] * NX;
      double n2 = 0.0;
      for (int le = 1 + lane_id(); le < len; le += NRTO_WAVE) {
        int k, x, b;
        entry_block<NX>(m, le, k, x, b);
        const double eta = (double)(r * fwd_gemm<NX, NU, F>(I, S, T, k, x, I.bvec + (int64_t)b * NU) + I.bhat[e0 + le]);
        n2 += eta * eta;
      }
      const double nrm = sqrt(wave_sum(n2));
      const double pi = I.C(CA_PI, c);
      // p~ = max(predicted p~, ||eta_j||): the cone point (p~, eta_j) is feasible
      const double pt = fmax(I.C(CA_PT, c), nrm);
      wave_sync();
      if (lane_id() == 0) {
        I.C(CA_PT, c) = pt;
        I.C(CA_PTT, c) = pt;
        I.C(CA_P, c) = pt;
      }
      for (int le = lane_id(); le < len; le += NRTO_WAVE) {
        if (le == 0) {
          I.st[e0] = (F)(pt + pi * inv_s);
        } else {
          int k, x, b;
          entry_block<NX>(m, le, k, x, b);
          const double eta = (double)(r * fwd_gemm<NX, NU, F>(I, S, T, k, x, I.bvec + (int64_t)b * NU) + I.bhat[e0 + le]);
          const double y = (nrm > 0.0) ? -pi * eta / nrm : 0.0;
          I.st[e0 + le] = (F)(eta + y * inv_s);
        }
      }
    }
  }
}


template <int NX, int NU, typename F>
__global__ void __launch_bounds__(NRTO_SOLVER_MAX_THREADS)
warm_kernel(DevPtrs g, SolveOpts o, const int32_t* order, int n, const float* pred, int64_t ld, int test,
            int32_t* accepted, double* res) {
  L<char>* smem = (L<char>*)nrto_dyn_smem;
  const int ii = order[blockIdx.x];
  Inst<NX, NU, F> I = make_inst<NX, NU, F>(g, ii);
  const int W = blockDim.x / NRTO_WAVE;
  Smem<F> S = carve<F>(smem, I.T, NX, NU, W);
  const int T = I.T;
  double r_cold = 1e300;
  cold_state<NX, NU, F, NRTO_DR>(I, S, o);
  if (test & 1) {
    load_kf<NX, NU, F>(I, S);
    r_cold = kkt_residual<NX, NU, F, NRTO_DR>(I, S, o, o.sigma_s, false, W);
  }
  // prediction row of this instance: du (T*NU), K (T*NU*NX as K[k][u][x]), p~ (ng), pi (ng).
  // The gains of the warm point stay those of the cold point (zero): a predicted
  // K with small errors along directions where every cone is slack would have to
  // be removed by the DR iteration's slowest mode.
  const float* pr = pred + (int64_t)ii * ld;
  for (int i = threadIdx.x; i < T * NU; i += blockDim.x) I.du[i] = (double)pr[i];
  pr += (test & 2) ? T * NU : T * NU * (NX + 1);   // bit 1: the row carries no gains
  for (int c = threadIdx.x; c < I.ng; c += blockDim.x) {
    const double pi = fmax(0.0, (double)pr[I.ng + c]);
    I.C(CA_PT, c) = (double)pr[c];   // the predicted p~, made cone-feasible by warm_pass
    I.C(CA_PI, c) = pi;
    I.C(CA_LAM, c) = -pi;
  }
  for (int i = threadIdx.x; i < T * NU * NX; i += blockDim.x) {
    I.K[i] = 0.0;
    I.Kt[i] = 0.0;
  }
  __syncthreads();
  load_kf<NX, NU, F>(I, S);
  if (wave_id() == 0) {
    rollout_dx<NX, NU, F>(I);
    const double psi = state_norm<NX, NU, F>(I);
    if (lane_id() == 0) I.iscr[ISCR_PSI] = psi;
  }
  if (threadIdx.x == 0) *S.ctr = 0;
  __syncthreads();
  warm_pass<NX, NU, F>(I, S, o);
  __syncthreads();
  double r_warm = 0.0;
  if (test & 1) r_warm = kkt_residual<NX, NU, F, NRTO_DR>(I, S, o, o.sigma_s, false, W);
  const bool keep = !(test & 1) || r_warm <= r_cold;
  if (!keep) cold_state<NX, NU, F, NRTO_DR>(I, S, o);
  if (threadIdx.x == 0) {
    accepted[ii] = keep ? 1 : 0;
    res[2 * ii] = r_warm;
    res[2 * ii + 1] = r_cold;
    g.rep[ii].sigma_s = o.sigma_s;   // the warm (or cold) point is built for the option's scaling
  }
}

template <int NX, int NU>
static hipError_t launch_warm_nxnu(const DevPtrs& g, const SolveOpts& o, const int32_t* order, int n, int threads,
                                   size_t smem, const float* pred, int64_t ld, int test, int32_t* acc, double* res,
                                   hipStream_t s) {
  dim3 grid(n), block(threads);
  if (o.precision == NRTO_FP32)
    hipLaunchKernelGGL((warm_kernel<NX, NU, float>), grid, block, smem, s, g, o, order, n, pred, ld, test, acc, res);
  else
    hipLaunchKernelGGL((warm_kernel<NX, NU, double>), grid, block, smem, s, g, o, order, n, pred, ld, test, acc, res);
  return hipGetLastError();
}

hipError_t launch_warm(const DevPtrs& g, const SolveOpts& o, int nx, const int32_t* order, int n, int threads,
                       size_t smem, const float* pred, int64_t ld, int test, int32_t* acc, double* res, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nx == 3) return launch_warm_nxnu<3, 2>(g, o, order, n, threads, smem, pred, ld, test, acc, res, s);
  if (nx == 12) return launch_warm_nxnu<12, 4>(g, o, order, n, threads, smem, pred, ld, test, acc, res, s);
  return launch_warm_nxnu<14, 7>(g, o, order, n, threads, smem, pred, ld, test, acc, res, s);
}

template <int NX, int NU, typename F, int METHOD>
__global__ void __launch_bounds__(NRTO_SOLVER_MAX_THREADS) solve_kernel(DevPtrs g, SolveOpts o, const int32_t* order, int n) {
  L<char>* smem = (L<char>*)nrto_dyn_smem;
  const int ii = order[blockIdx.x];
  solve_instance<NX, NU, F, METHOD>(g, o, ii, smem);
}

size_t solver_smem_bytes(int T, int nx, int nu, int precision, int threads) {
  return smem_bytes(T, nx, nu, precision == NRTO_FP32 ? 4 : 8, threads / NRTO_WAVE);
}

template <int NX, int NU>
static hipError_t launch_nxnu(const DevPtrs& g, const SolveOpts& o, const int32_t* order, int n, int threads,
                              size_t smem, hipStream_t s) {
  dim3 grid(n), block(threads);
  if (o.precision == NRTO_FP32) {
    if (o.method == NRTO_DR)
      hipLaunchKernelGGL((solve_kernel<NX, NU, float, NRTO_DR>), grid, block, smem, s, g, o, order, n);
    else
      hipLaunchKernelGGL((solve_kernel<NX, NU, float, NRTO_FULLADMM>), grid, block, smem, s, g, o, order, n);
  } else {
    if (o.method == NRTO_DR)
      hipLaunchKernelGGL((solve_kernel<NX, NU, double, NRTO_DR>), grid, block, smem, s, g, o, order, n);
    else
      hipLaunchKernelGGL((solve_kernel<NX, NU, double, NRTO_FULLADMM>), grid, block, smem, s, g, o, order, n);
  }
  return hipGetLastError();
}

// One launch per dynamics model present; `order` lists the instances of that
// model (largest first).
hipError_t launch_solver(const DevPtrs& g, const SolveOpts& o, int nx, const int32_t* order, int n, int threads,
                         size_t smem, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nx == 3) return launch_nxnu<3, 2>(g, o, order, n, threads, smem, s);
  if (nx == 12) return launch_nxnu<12, 4>(g, o, order, n, threads, smem, s);
  return launch_nxnu<14, 7>(g, o, order, n, threads, smem, s);
}

template <int NX, int NU>
static hipError_t smem_attr(size_t bytes) {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)warm_kernel<NX, NU, float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)warm_kernel<NX, NU, double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)solve_kernel<NX, NU, float, NRTO_DR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)solve_kernel<NX, NU, float, NRTO_FULLADMM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)solve_kernel<NX, NU, double, NRTO_DR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)solve_kernel<NX, NU, double, NRTO_FULLADMM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t set_solver_smem_limit(size_t bytes) {
  hipError_t e = smem_attr<3, 2>(bytes);
  if (e != hipSuccess) return e;
  e = smem_attr<12, 4>(bytes);
  if (e != hipSuccess) return e;
  return smem_attr<14, 7>(bytes);
}

}  // namespace nrto
