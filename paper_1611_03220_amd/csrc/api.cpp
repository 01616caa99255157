// C ABI of libkrr: argument checks, workspace layout, and the PCG driver (Alg. 1).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/krr.h"
#include "kernels.hpp"

using namespace krr;

namespace {

thread_local char g_err[512] = "";

krr_status fail(krr_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define CHECK_HIP(...)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (__VA_ARGS__);                                                        \
    if (e_ != hipSuccess)                                                                 \
      return fail(KRR_E_HIP, "%s failed: %s (line %d)", #__VA_ARGS__, hipGetErrorString(e_), \
                  __LINE__);                                                              \
  } while (0)

#define CHECK_ST(expr)                     \
  do {                                     \
    krr_status s_ = (expr);                \
    if (s_ != KRR_OK) return s_;           \
  } while (0)

// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base(static_cast<char*>(b)) {}
  template <typename T> T* take(int64_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    return p;
  }
};

constexpr int NBLK = 256;  // blocks of the column-wise reductions

bool prec_ok(int32_t p) { return p == KRR_PREC_FP64 || p == KRR_PREC_F16X3 || p == KRR_PREC_BF16X3; }

int64_t kp_for(int64_t d) { return round_up(d + 2, K_STEP); }
// The F16X3 product uses MFMA accumulation (up to 32 columns of V per pass) for every d;
// the BF16X3 product keeps the VALU-accumulate kernel.
// (d + 3 <= 128: row operands in registers; larger d: both operands through LDS)
bool use_pv(int prec, int64_t d) { return prec == KRR_PREC_F16X3; }
int64_t kp_for(int prec, int64_t d) {
  return use_pv(prec, d) ? round_up(d + 2 + (PSHIFT > 0), K_STEP) : kp_for(d);
}
// FP64 point width: multiples of 8 up to 128 (FP64 MFMA kernel), else of 32 (VALU kernel)
int64_t dp_for(int64_t d) { return round_up(d, 8) <= 128 ? round_up(d, 8) : round_up(d, 32); }

// Split of the column sweep over blockIdx.y so that small row counts still fill the chip.
int choose_nsplit(int64_t n1, int64_t n2) {
  const int64_t rowblocks = ceil_div(n1, 128);
  const int64_t tiles = ceil_div(n2, 64);
  int64_t ns = ceil_div(2048, rowblocks);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, tiles / 4));
  return (int)std::max<int64_t>(1, std::min<int64_t>(ns, 64));
}

// --------------------------------------------------------- kernel-product context
struct MatmatCtx {
  int prec = KRR_PREC_F16X3;
  bool pv = false;          // MFMA-accumulate kernel
  _Float16 *Vth = nullptr, *Vtl = nullptr;  // [mpad][rp2] split V^T (pv)
  float *colmax = nullptr, *vscale = nullptr;
  int64_t mpad = 0;
  int64_t n1 = 0, n2 = 0, d = 0, m = 0;
  int64_t rp1 = 0, rp2 = 0, Kp = 0, dp = 0;
  int nsplit = 1;
  float* stats = nullptr;   // [0] max|x|, [1] max nu, [2] 1/q^2
  void *Ahi = nullptr, *Alo = nullptr, *Bhi = nullptr, *Blo = nullptr;
  double *XA = nullptr, *nuA = nullptr, *XB = nullptr, *nuB = nullptr;
  double* part = nullptr;   // nsplit x rp1 x m
  int64_t part_stride = 0;
  double c2 = 0;            // log2(e) / (2 sigma^2)
  double sigma = 0;
};

void layout_matmat(Bump& b, MatmatCtx& c, int64_t n1, int64_t n2, int64_t d, int64_t m, int prec,
                   bool square) {
  c.prec = prec;
  c.n1 = n1; c.n2 = n2; c.d = d; c.m = m;
  c.rp1 = round_up(n1, ROW_PAD);
  c.rp2 = round_up(n2, ROW_PAD);
  c.nsplit = choose_nsplit(n1, n2);
  c.stats = b.take<float>(64);
  if (prec == KRR_PREC_FP64) {
    c.dp = dp_for(d);
    c.XA = b.take<double>(c.rp1 * c.dp);
    c.nuA = b.take<double>(c.rp1);
    if (square) { c.XB = c.XA; c.nuB = c.nuA; }
    else { c.XB = b.take<double>(c.rp2 * c.dp); c.nuB = b.take<double>(c.rp2); }
  } else {
    c.pv = use_pv(prec, d);
    c.Kp = kp_for(prec, d);
    if (c.pv) {
      c.mpad = round_up(std::min<int64_t>(m, 32), 16);
      c.Vth = b.take<_Float16>(c.mpad * c.rp2);
      c.Vtl = b.take<_Float16>(c.mpad * c.rp2);
      c.colmax = b.take<float>(m);
      c.vscale = b.take<float>(c.mpad);
    }
    c.Ahi = b.take<uint16_t>(c.rp1 * c.Kp);
    c.Alo = b.take<uint16_t>(c.rp1 * c.Kp);
    c.Bhi = b.take<uint16_t>(c.rp2 * c.Kp);
    c.Blo = b.take<uint16_t>(c.rp2 * c.Kp);
  }
  c.part_stride = c.rp1 * m;
  c.part = b.take<double>(c.nsplit * c.part_stride);
}

// Prepare both point sets for a given sigma (X2 == nullptr: square product of X1).
hipError_t prepare_points(MatmatCtx& c, const float* X1, int64_t ldx1, const float* X2,
                          int64_t ldx2, double sigma, hipStream_t st) {
  c.sigma = sigma;
  c.c2 = 1.4426950408889634 / (2.0 * sigma * sigma);
  hipError_t e;
  if (c.prec == KRR_PREC_FP64) {
    if ((e = prep_points_f64(X1, c.n1, c.d, ldx1, c.rp1, c.dp, c.XA, c.nuA, st))) return e;
    if (X2 && (e = prep_points_f64(X2, c.n2, c.d, ldx2, c.rp2, c.dp, c.XB, c.nuB, st))) return e;
    return hipSuccess;
  }
  if ((e = fill_f32(c.stats, 4, 0.0f, st))) return e;
  if ((e = point_stats(X1, c.n1, c.d, ldx1, c.stats, st))) return e;
  if (X2 && (e = point_stats(X2, c.n2, c.d, ldx2, c.stats, st))) return e;
  const float* Xb = X2 ? X2 : X1;
  const int64_t ldb = X2 ? ldx2 : ldx1;
  const int ps = c.pv ? PSHIFT : 0;
  if (c.prec == KRR_PREC_F16X3) {
    if ((e = prep_points<_Float16>(X1, c.n1, c.d, ldx1, c.rp1, c.Kp, c.c2, c.stats, 0, ps,
                                   (_Float16*)c.Ahi, (_Float16*)c.Alo, c.stats + 2, st)))
      return e;
    return prep_points<_Float16>(Xb, c.n2, c.d, ldb, c.rp2, c.Kp, c.c2, c.stats, 1, ps,
                                 (_Float16*)c.Bhi, (_Float16*)c.Blo, nullptr, st);
  }
  if ((e = prep_points<__bf16>(X1, c.n1, c.d, ldx1, c.rp1, c.Kp, c.c2, c.stats, 0, 0,
                               (__bf16*)c.Ahi, (__bf16*)c.Alo, c.stats + 2, st)))
    return e;
  return prep_points<__bf16>(Xb, c.n2, c.d, ldb, c.rp2, c.Kp, c.c2, c.stats, 1, 0, (__bf16*)c.Bhi,
                             (__bf16*)c.Blo, nullptr, st);
}

// Partial sums of K V (or dK/dsigma V) into c.part. V is FP32 (mixed) or FP64 (FP64 path).
// On the MFMA-accumulate path Vf (n2 x ldv) is split in place: on return it holds exactly the
// vector the product used.
hipError_t run_matmat(const MatmatCtx& c, float* Vf, const double* V64, int64_t ldv, bool deriv,
                      hipStream_t st) {
  const double sig3 = c.sigma * c.sigma * c.sigma;
  if (c.prec == KRR_PREC_FP64) {
    F64Points A{c.XA, c.nuA, c.n1, c.dp}, B{c.XB, c.nuB, c.n2, c.dp};
    return matmat_f64(A, B, V64, ldv, c.m, deriv, 1.0 / (2.0 * c.sigma * c.sigma), 1.0 / sig3,
                      c.part, c.m, c.part_stride, c.nsplit, st);
  }
  const float dscale = (float)(1.0 / (c.c2 * sig3));  // dk/dsigma = k * (-log2 k) / (c2 sigma^3)
  if (c.prec == KRR_PREC_F16X3) {
    MixedPoints<_Float16> A{(const _Float16*)c.Ahi, (const _Float16*)c.Alo, c.n1, c.Kp, c.stats + 2};
    MixedPoints<_Float16> B{(const _Float16*)c.Bhi, (const _Float16*)c.Blo, c.n2, c.Kp, c.stats + 2};
    if (c.pv) {
      for (int64_t c0 = 0; c0 < c.m; c0 += 32) {
        const int64_t mc = std::min<int64_t>(32, c.m - c0);
        const int64_t mp = round_up(mc, 16);
        hipError_t e = vec_split_t(Vf + c0, c.n2, mc, ldv, c.rp2, mp, c.colmax, PSHIFT, c.Vth,
                                   c.Vtl, c.vscale, st);
        if (e != hipSuccess) return e;
        SplitRhs V{c.Vth, c.Vtl, c.vscale, c.rp2, mp};
        e = matmat_f16pv(A, B, V, mc, deriv, dscale, c.part + c0, c.m, c.part_stride, c.nsplit, st);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
    return matmat_mixed<_Float16>(A, B, Vf, ldv, c.m, deriv, dscale, c.part, c.m, c.part_stride,
                                  c.nsplit, st);
  }
  MixedPoints<__bf16> A{(const __bf16*)c.Ahi, (const __bf16*)c.Alo, c.n1, c.Kp, c.stats + 2};
  MixedPoints<__bf16> B{(const __bf16*)c.Bhi, (const __bf16*)c.Blo, c.n2, c.Kp, c.stats + 2};
  return matmat_mixed<__bf16>(A, B, Vf, ldv, c.m, deriv, dscale, c.part, c.m, c.part_stride,
                              c.nsplit, st);
}

krr_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws) return fail(KRR_E_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(KRR_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(KRR_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return KRR_OK;
}

// ------------------------------------------------------------------ features
struct FeatLayout {
  float* stats;
  _Float16 *Xh, *Xl, *Wh, *Wl;
  int64_t dk, np, sp;
};
void layout_features(Bump& b, FeatLayout& L, int64_t n, int64_t d, int64_t s) {
  L.dk = round_up(d, 32);
  L.np = round_up(n, 64);
  L.sp = round_up(s, 64);
  L.stats = b.take<float>(64);
  L.Xh = b.take<_Float16>(L.np * L.dk);
  L.Xl = b.take<_Float16>(L.np * L.dk);
  L.Wh = b.take<_Float16>(L.sp * L.dk);
  L.Wl = b.take<_Float16>(L.sp * L.dk);
}

// ---------------------------------------------------------------- precond factor
int64_t pow2_pad(int64_t s) {
  int64_t p = 64;
  while (p < s) p *= 2;
  return p;
}
int gram_nsplit(int64_t s, int64_t n) {
  const int64_t t = ceil_div(s, 64);
  const int64_t tiles = t * (t + 1) / 2;
  int64_t ns = ceil_div(2048, tiles);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, ceil_div(n, 2048)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(ns, 32));
}
struct FactorLayout {
  float* stats;
  _Float16 *h1, *l1;     // Zt split (sp64 x nk), later Z split (np x sk)
  _Float16 *ch, *cl;     // Cinv split (sp64 x sk)
  double *part, *G, *Cinv, *tmp;
  int* info;
  int64_t nk, sk, np, sp64, s_pad;
  int nsplit;
};
void layout_factor(Bump& b, FactorLayout& L, int64_t n, int64_t s) {
  L.nk = round_up(n, 32);
  L.sk = round_up(s, 32);
  L.np = round_up(n, 64);
  L.sp64 = round_up(s, 64);
  L.s_pad = pow2_pad(s);
  L.nsplit = gram_nsplit(s, n);
  L.stats = b.take<float>(64);
  L.info = b.take<int>(64);
  const int64_t big = std::max(L.sp64 * L.nk, L.np * L.sk);
  L.h1 = b.take<_Float16>(big);
  L.l1 = b.take<_Float16>(big);
  L.ch = b.take<_Float16>(L.sp64 * L.sk);
  L.cl = b.take<_Float16>(L.sp64 * L.sk);
  L.part = b.take<double>((int64_t)L.nsplit * s * s);
  L.G = b.take<double>(L.s_pad * L.s_pad);
  L.Cinv = b.take<double>(L.s_pad * L.s_pad);
  L.tmp = b.take<double>(L.s_pad * L.s_pad / 2);
}

// ---------------------------------------------------------------------- PCG
struct PCGLayout {
  MatmatCtx mm;      // kernel product in the solve precision
  MatmatCtx mm64;    // FP64 product for the true residual / refinement
  float* pf;         // FP32 copy of p (mixed)
  double *p, *q, *r, *z, *ax, *delta, *rhs;
  double *part_yy, *part_rr, *part_pq, *part_rz, *pc_part, *T;
  double *ynorm, *rnorm, *rho, *alpha, *beta, *hist;
  int *active, *broken, *col_iters, *count;
  int nchunk;
};
int precond_nchunk(int64_t n, int64_t s) {
  const int64_t kb = ceil_div(std::max<int64_t>(s, 1), 256);
  int64_t nc = ceil_div(1024, kb);
  nc = std::min<int64_t>(nc, std::max<int64_t>(1, ceil_div(n, 256)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(nc, 512));
}
void layout_pcg(Bump& b, PCGLayout& L, int64_t n, int64_t d, int64_t s, int64_t m, int prec) {
  layout_matmat(b, L.mm, n, n, d, m, prec, true);
  if (prec != KRR_PREC_FP64) layout_matmat(b, L.mm64, n, n, d, m, KRR_PREC_FP64, true);
  const int64_t nm = n * m;
  L.pf = b.take<float>(round_up(n, ROW_PAD) * m);
  L.p = b.take<double>(nm);
  L.q = b.take<double>(nm);
  L.r = b.take<double>(nm);
  L.z = b.take<double>(nm);
  L.ax = b.take<double>(nm);
  L.delta = b.take<double>(nm);
  L.rhs = b.take<double>(nm);
  L.part_yy = b.take<double>(NBLK * m);
  L.part_rr = b.take<double>(NBLK * m);
  L.part_pq = b.take<double>(NBLK * m);
  L.part_rz = b.take<double>(NBLK * m);
  L.nchunk = precond_nchunk(n, s);
  L.pc_part = b.take<double>((int64_t)L.nchunk * std::max<int64_t>(s, 1) * m);
  L.T = b.take<double>(std::max<int64_t>(s, 1) * m);
  L.ynorm = b.take<double>(m);
  L.rnorm = b.take<double>(m);
  L.rho = b.take<double>(m);
  L.alpha = b.take<double>(m);
  L.beta = b.take<double>(m);
  L.hist = b.take<double>(2);
  L.active = b.take<int>(m);
  L.broken = b.take<int>(m);
  L.col_iters = b.take<int>(m);
  L.count = b.take<int>(2);
}

struct GradLayout {
  MatmatCtx mm;
  float* af;   // FP32 copy of alpha for the mixed product
  double* w;
  double* part;
};
void layout_grad(Bump& b, GradLayout& L, int64_t n, int64_t d, int64_t m, int prec) {
  layout_matmat(b, L.mm, n, n, d, m, prec, true);
  L.af = b.take<float>(round_up(n, ROW_PAD) * m);
  L.w = b.take<double>(n * m);
  L.part = b.take<double>(NBLK * m * 2);
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* krr_last_error(void) { return g_err; }
const char* krr_version(void) { return "libkrr 0.1 (gfx950)"; }

void krr_pcg_defaults(krr_pcg_opts* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->max_iter = 1000;
  o->prec = KRR_PREC_F16X3;
  o->use_precond = 1;
  o->check_every = 1;
  o->lambda_p = 0.0;
  o->true_residual = 1;
  o->refine = 0;
  o->warm_start = 0;
}

size_t krr_workspace_bytes(int32_t op, int64_t n1, int64_t n2, int64_t d, int64_t s, int64_t m,
                           int32_t prec) {
  if (n1 < 1 || d < 0 || s < 0 || m < 0) return 0;
  if (!prec_ok(prec)) prec = KRR_PREC_F16X3;
  Bump b(nullptr);
  switch (op) {
    case KRR_OP_FEATURES: { FeatLayout L; layout_features(b, L, n1, d, s); break; }
    case KRR_OP_PRECOND_FACTOR: { FactorLayout L; layout_factor(b, L, n1, s); break; }
    case KRR_OP_KERNEL_MATMAT: {
      MatmatCtx c;
      layout_matmat(b, c, n1, n2, d, m, prec, false);
      if (prec != KRR_PREC_FP64) b.take<float>(round_up(n2, ROW_PAD) * m);
      break;
    }
    case KRR_OP_PCG_SOLVE: { PCGLayout L; layout_pcg(b, L, n1, d, s, m, prec); break; }
    case KRR_OP_GRAD: { GradLayout L; layout_grad(b, L, n1, d, m, prec); break; }
    default: return 0;
  }
  return b.off + 256;
}

// ------------------------------------------------------------------ features
krr_status krr_features(const float* X, int64_t n, int64_t d, int64_t ldx, const float* W,
                        const float* b, int64_t s, float* Z, int64_t ldz, void* ws,
                        size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X || !W || !b || !Z) return fail(KRR_E_ARG, "krr_features: null pointer");
  if (n < 1 || d < 1 || s < 1 || ldx < d || ldz < s)
    return fail(KRR_E_ARG, "krr_features: bad sizes n=%lld d=%lld s=%lld", (long long)n,
                (long long)d, (long long)s);
  Bump probe(nullptr);
  FeatLayout L;
  layout_features(probe, L, n, d, s);
  CHECK_ST(check_ws(ws, ws_bytes, probe.off + 256));
  Bump bb(ws);
  layout_features(bb, L, n, d, s);
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(fill_f32(L.stats, 4, 0.0f, st));
  CHECK_HIP(absmax<float>(X, n, d, ldx, L.stats + 0, st));
  CHECK_HIP(absmax<float>(W, d, s, s, L.stats + 1, st));
  CHECK_HIP((split_operand<float, _Float16>(X, n, d, ldx, L.stats + 0, 0, L.np, L.dk, L.Xh, L.Xl, st)));
  // W is d x s; its transpose (s x d, contraction index contiguous) is the B operand
  CHECK_HIP((split_operand<float, _Float16>(W, d, s, s, L.stats + 1, 1, L.sp, L.dk, L.Wh, L.Wl, st)));
  SplitOperand A{L.Xh, L.Xl, L.dk, L.stats + 0}, B{L.Wh, L.Wl, L.dk, L.stats + 1};
  CHECK_HIP(gemm_nt_f16x3(A, B, n, s, L.dk, 1, EPI_COS, 0, 0, 1.0, nullptr, 0, Z, ldz, b,
                          (float)std::sqrt(2.0 / (double)s), st));
  return KRR_OK;
}

// ---------------------------------------------------------------- precond factor
krr_status krr_precond_factor(const float* Z, int64_t n, int64_t s, int64_t ldz, double lambda_p,
                              double* C, float* Ut, int64_t ldu, void* ws, size_t ws_bytes,
                              int64_t* info, void* stream) {
  g_err[0] = 0;
  if (!Z || !C || !Ut || !info) return fail(KRR_E_ARG, "krr_precond_factor: null pointer");
  *info = 0;
  if (n < 2 || s < 1 || s >= n || ldz < s || ldu < s)
    return fail(KRR_E_ARG, "krr_precond_factor: need 1 <= s < n and ld >= s (n=%lld s=%lld)",
                (long long)n, (long long)s);
  if (!(lambda_p > 0.0) || !std::isfinite(lambda_p))
    return fail(KRR_E_ARG, "krr_precond_factor: lambda_p must be > 0");
  Bump probe(nullptr);
  FactorLayout L;
  layout_factor(probe, L, n, s);
  CHECK_ST(check_ws(ws, ws_bytes, probe.off + 256));
  Bump bb(ws);
  layout_factor(bb, L, n, s);
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(fill_f32(L.stats, 4, 0.0f, st));
  CHECK_HIP(fill_i32(L.info, 1, 0, st));
  // Gram G = Z^T Z: A = B = Z^T (s x n, contraction over points)
  CHECK_HIP(absmax<float>(Z, n, s, ldz, L.stats + 0, st));
  CHECK_HIP((split_operand<float, _Float16>(Z, n, s, ldz, L.stats + 0, 1, L.sp64, L.nk, L.h1, L.l1, st)));
  SplitOperand Zt{L.h1, L.l1, L.nk, L.stats + 0};
  CHECK_HIP(gemm_nt_f16x3(Zt, Zt, s, s, L.nk, L.nsplit, EPI_PART64, 1, 0, 1.0, L.part, s * s,
                          nullptr, s, nullptr, 0.0f, st));
  CHECK_HIP(gram_finalize(L.part, L.nsplit, s, s, s * s, lambda_p, L.s_pad, L.G, st));
  // Cholesky (FP64) and inverse of the factor
  CHECK_HIP(fill_f64(L.Cinv, L.s_pad * L.s_pad, 0.0, st));
  CHECK_HIP(cholesky_blocked(L.G, L.s_pad, L.Cinv, L.info, st));
  int hinfo = 0;
  CHECK_HIP(hipMemcpyAsync(&hinfo, L.info, sizeof(int), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  if (hinfo != 0) {
    *info = hinfo;
    return fail(KRR_E_NOT_SPD, "krr_precond_factor: Z^T Z + lambda_p I not positive definite at pivot %d", hinfo);
  }
  CHECK_HIP(tri_inverse_doubling(L.G, L.s_pad, L.Cinv, L.tmp, st));
  CHECK_HIP(copy_lower(L.G, L.s_pad, s, C, st));
  // Ut = Z C^{-T}: A = Z (n x s), B = C^{-1} (rows j, contraction k), lower triangular
  CHECK_HIP(absmax<double>(L.Cinv, s, s, L.s_pad, L.stats + 1, st));
  CHECK_HIP((split_operand<float, _Float16>(Z, n, s, ldz, L.stats + 0, 0, L.np, L.sk, L.h1, L.l1, st)));
  CHECK_HIP((split_operand<double, _Float16>(L.Cinv, s, s, L.s_pad, L.stats + 1, 0, L.sp64, L.sk, L.ch, L.cl, st)));
  SplitOperand A{L.h1, L.l1, L.sk, L.stats + 0}, B{L.ch, L.cl, L.sk, L.stats + 1};
  CHECK_HIP(gemm_nt_f16x3(A, B, n, s, L.sk, 1, EPI_F32, 0, 1, 1.0, nullptr, 0, Ut, ldu, nullptr,
                          0.0f, st));
  CHECK_HIP(hipStreamSynchronize(st));
  return KRR_OK;
}

// ---------------------------------------------------------------- kernel matmat
krr_status krr_kernel_matmat(const float* X1, int64_t n1, int64_t ldx1, const float* X2, int64_t n2,
                             int64_t ldx2, int64_t d, double sigma, double shift, const double* V,
                             int64_t m, int64_t ldv, double* OUT, int64_t ldo, int32_t deriv,
                             int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X1 || !X2 || !V || !OUT) return fail(KRR_E_ARG, "krr_kernel_matmat: null pointer");
  if (n1 < 1 || n2 < 1 || d < 1 || m < 1 || ldx1 < d || ldx2 < d || ldv < m || ldo < m)
    return fail(KRR_E_ARG, "krr_kernel_matmat: bad sizes or strides");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(KRR_E_ARG, "krr_kernel_matmat: sigma must be > 0");
  if (shift != 0.0 && n1 != n2) return fail(KRR_E_ARG, "krr_kernel_matmat: shift needs n1 == n2");
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "krr_kernel_matmat: unknown precision %d", prec);
  if (prec == KRR_PREC_BF16X3 && kp_for(d) > 256)
    return fail(KRR_E_ARG, "krr_kernel_matmat: BF16X3 supports d <= 254 (d=%lld)", (long long)d);
  const size_t need = krr_workspace_bytes(KRR_OP_KERNEL_MATMAT, n1, n2, d, 0, m, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  MatmatCtx c;
  layout_matmat(bb, c, n1, n2, d, m, prec, false);
  float* Vf = prec != KRR_PREC_FP64 ? bb.take<float>(round_up(n2, ROW_PAD) * m) : nullptr;
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(prepare_points(c, X1, ldx1, X2, ldx2, sigma, st));
  if (Vf) {
    CHECK_HIP(vec_to_f32(V, n2, m, ldv, round_up(n2, ROW_PAD), m, Vf, st));
    CHECK_HIP(run_matmat(c, Vf, nullptr, m, deriv != 0, st));
  } else {
    CHECK_HIP(run_matmat(c, nullptr, V, ldv, deriv != 0, st));
  }
  CHECK_HIP(matmat_finalize<double>(c.part, c.part_stride, c.nsplit, n1, m, m, shift, V, ldv, OUT,
                                    ldo, st));
  return KRR_OK;
}

// ------------------------------------------------------------------------ PCG
namespace {

// Device time of the kernel products of one solve: HIP event pairs on the solve's stream,
// harvested at synchronisation points.
struct MMTimer {
  static constexpr int CAP = 32;
  hipEvent_t a[CAP], b[CAP];
  int used = 0, created = 0, calls = 0;
  double ms = 0.0;
  hipError_t init() {
    for (; created < CAP; ++created) {
      hipError_t e = hipEventCreate(&a[created]);
      if (e != hipSuccess) return e;
      e = hipEventCreate(&b[created]);
      if (e != hipSuccess) { (void)hipEventDestroy(a[created]); return e; }
    }
    return hipSuccess;
  }
  ~MMTimer() {
    for (int i = 0; i < created; ++i) { (void)hipEventDestroy(a[i]); (void)hipEventDestroy(b[i]); }
  }
  hipError_t harvest() {
    if (used == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(b[used - 1]);
    if (e != hipSuccess) return e;
    for (int i = 0; i < used; ++i) {
      float t = 0.0f;
      if ((e = hipEventElapsedTime(&t, a[i], b[i])) != hipSuccess) return e;
      ms += t;
    }
    used = 0;
    return hipSuccess;
  }
  hipError_t begin(hipStream_t st) {
    if (used == CAP) {
      hipError_t e = harvest();
      if (e != hipSuccess) return e;
    }
    return hipEventRecord(a[used], st);
  }
  hipError_t end(hipStream_t st) {
    hipError_t e = hipEventRecord(b[used], st);
    ++used;
    ++calls;
    return e;
  }
};

hipError_t timed_matmat(MMTimer* tm, const MatmatCtx& c, float* Vf, const double* V64,
                        int64_t ldv, bool deriv, hipStream_t st) {
  hipError_t e;
  if (tm && (e = tm->begin(st)) != hipSuccess) return e;
  if ((e = run_matmat(c, Vf, V64, ldv, deriv, st)) != hipSuccess) return e;
  return tm ? tm->end(st) : hipSuccess;
}

hipError_t fill2d_zero(double* a, int64_t lda, int64_t n, int64_t m, hipStream_t st) {
  if (lda == m) return fill_f64(a, n * m, 0.0, st);
  for (int64_t i = 0; i < n; ++i) {  // strided: one small fill per row is acceptable here
    hipError_t e = fill_f64(a + i * lda, m, 0.0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct SolveArgs {
  PCGLayout* L;
  int64_t n, m, s, ldu;
  const float* Ut;
  double lambda, lambda_p, tol;
  int use_precond, max_iter, check_every;
  bool mixed;
  MMTimer* tm;
};

// One PCG run on A x = rhs (rhs n x m contiguous, x strided), starting from x.
// warm: x holds a starting point that is not zero. Returns iterations through *iters.
krr_status pcg_core(const SolveArgs& a, const double* rhs, int64_t ldr, double* x, int64_t ldx,
                    bool warm, int* iters, std::vector<double>* hist, hipStream_t st) {
  PCGLayout& L = *a.L;
  const int64_t n = a.n, m = a.m;
  CGScalars S{L.ynorm, L.rnorm, L.rho, L.alpha, L.beta, L.active, L.broken, L.col_iters, L.count};
  const int64_t ldpf = m;
  // r0 = rhs - A x0
  if (warm) {
    if (a.mixed) {
      CHECK_HIP(fill_f32(L.pf, round_up(n, ROW_PAD) * m, 0.0f, st));
      // FP32 copy of x for the product (row stride m)
      CHECK_HIP(copy2d(x, ldx, L.p, m, n, m, st));
      CHECK_HIP(cg_update_p(L.p, L.p, L.pf, ldpf, L.beta, L.active, 1, n, m, st));
      CHECK_HIP(timed_matmat(a.tm, L.mm, L.pf, nullptr, ldpf, false, st));
    } else {
      CHECK_HIP(copy2d(x, ldx, L.p, m, n, m, st));
      CHECK_HIP(timed_matmat(a.tm, L.mm, nullptr, L.p, m, false, st));
    }
    CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, a.lambda,
                                      L.p, m, L.ax, m, st));
    CHECK_HIP(residual_from(rhs, ldr, L.ax, n, m, L.r, st));
  } else {
    CHECK_HIP(residual_from(rhs, ldr, nullptr, n, m, L.r, st));
  }
  CHECK_HIP(dot_partial<double, double>(rhs, ldr, rhs, ldr, n, m, L.part_yy, NBLK, st));
  CHECK_HIP(dot_partial<double, double>(L.r, m, L.r, m, n, m, L.part_rr, NBLK, st));
  if (a.use_precond) {
    CHECK_HIP(precond_apply(a.Ut, a.ldu, n, a.s, m, a.lambda_p, L.r, L.z, L.pc_part, L.nchunk, L.T, st));
    CHECK_HIP(dot_partial<double, double>(L.r, m, L.z, m, n, m, L.part_rz, NBLK, st));
  } else {
    CHECK_HIP(copy2d(L.r, m, L.z, m, n, m, st));
  }
  CHECK_HIP(cg_init_scalars(L.part_yy, L.part_rr, a.use_precond ? L.part_rz : nullptr, NBLK, m,
                            a.tol, S, st));
  CHECK_HIP(cg_update_p(L.z, L.p, a.mixed ? L.pf : nullptr, ldpf, L.beta, L.active, 1, n, m, st));
  int h_count = 0;
  CHECK_HIP(hipMemcpyAsync(&h_count, L.count, sizeof(int), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  int it = 0;
  while (h_count > 0 && it < a.max_iter) {
    ++it;
    // q = (K + lambda I) p
    if (a.mixed) {
      CHECK_HIP(timed_matmat(a.tm, L.mm, L.pf, nullptr, ldpf, false, st));
      CHECK_HIP(matmat_finalize<float>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, a.lambda,
                                       L.pf, ldpf, L.q, m, st));
      CHECK_HIP(dot_partial<float, double>(L.pf, ldpf, L.q, m, n, m, L.part_pq, NBLK, st));
    } else {
      CHECK_HIP(timed_matmat(a.tm, L.mm, nullptr, L.p, m, false, st));
      CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, a.lambda,
                                        L.p, m, L.q, m, st));
      CHECK_HIP(dot_partial<double, double>(L.p, m, L.q, m, n, m, L.part_pq, NBLK, st));
    }
    CHECK_HIP(cg_alpha(L.part_pq, NBLK, m, S, st));
    if (a.mixed)
      CHECK_HIP(cg_update_xr<float>(x, ldx, L.r, L.pf, ldpf, L.q, L.alpha, n, m, L.part_rr, NBLK, st));
    else
      CHECK_HIP(cg_update_xr<double>(x, ldx, L.r, L.p, m, L.q, L.alpha, n, m, L.part_rr, NBLK, st));
    CHECK_HIP(cg_conv(L.part_rr, NBLK, m, a.tol, it, S, L.hist, st));
    if (a.use_precond) {
      CHECK_HIP(precond_apply(a.Ut, a.ldu, n, a.s, m, a.lambda_p, L.r, L.z, L.pc_part, L.nchunk, L.T, st));
      CHECK_HIP(dot_partial<double, double>(L.r, m, L.z, m, n, m, L.part_rz, NBLK, st));
      CHECK_HIP(cg_beta(L.part_rz, nullptr, NBLK, m, S, st));
      CHECK_HIP(cg_update_p(L.z, L.p, a.mixed ? L.pf : nullptr, ldpf, L.beta, L.active, 0, n, m, st));
    } else {
      CHECK_HIP(cg_beta(nullptr, L.part_rr, NBLK, m, S, st));
      CHECK_HIP(cg_update_p(L.r, L.p, a.mixed ? L.pf : nullptr, ldpf, L.beta, L.active, 0, n, m, st));
    }
    if (it % a.check_every == 0 || it == a.max_iter) {
      double hv = 0.0;
      CHECK_HIP(hipMemcpyAsync(&h_count, L.count, sizeof(int), hipMemcpyDeviceToHost, st));
      CHECK_HIP(hipMemcpyAsync(&hv, L.hist, sizeof(double), hipMemcpyDeviceToHost, st));
      CHECK_HIP(hipStreamSynchronize(st));
      if (hist) hist->push_back(hv);
    }
  }
  *iters = it;
  return KRR_OK;
}

// FP64 true residual R = rhs - (K + lambda I) x into L.ax; per-column relative norms to host.
krr_status true_residual(PCGLayout& L, const SolveArgs& a, const double* Y, int64_t ldy,
                         const double* x, int64_t ldx, std::vector<double>& rel, hipStream_t st) {
  MatmatCtx& c = a.mixed ? L.mm64 : L.mm;
  const int64_t n = a.n, m = a.m;
  CHECK_HIP(copy2d(x, ldx, L.delta, m, n, m, st));
  CHECK_HIP(run_matmat(c, nullptr, L.delta, m, false, st));  // FP64 check: not timed
  CHECK_HIP(matmat_finalize<double>(c.part, c.part_stride, c.nsplit, n, m, m, a.lambda, L.delta, m,
                                    L.ax, m, st));
  CHECK_HIP(residual_from(Y, ldy, L.ax, n, m, L.rhs, st));
  CHECK_HIP(dot_partial<double, double>(L.rhs, m, L.rhs, m, n, m, L.part_rr, NBLK, st));
  CHECK_HIP(dot_partial<double, double>(Y, ldy, Y, ldy, n, m, L.part_yy, NBLK, st));
  std::vector<double> prr(NBLK * m), pyy(NBLK * m);
  CHECK_HIP(hipMemcpyAsync(prr.data(), L.part_rr, sizeof(double) * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipMemcpyAsync(pyy.data(), L.part_yy, sizeof(double) * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  rel.assign(m, 0.0);
  for (int64_t c2 = 0; c2 < m; ++c2) {
    double rr = 0.0, yy = 0.0;
    for (int b = 0; b < NBLK; ++b) { rr += prr[b * m + c2]; yy += pyy[b * m + c2]; }
    rel[c2] = yy > 0.0 ? std::sqrt(rr) / std::sqrt(yy) : std::sqrt(rr);
  }
  return KRR_OK;
}

}  // namespace

krr_status krr_pcg_solve(const float* X, int64_t n, int64_t d, int64_t ldx, double sigma,
                         double lambda, const float* Ut, int64_t s, int64_t ldu, const double* Y,
                         int64_t ldy, double* alpha, int64_t lda, int64_t m,
                         const krr_pcg_opts* opts, krr_pcg_report* rep, void* ws, size_t ws_bytes,
                         void* stream) {
  g_err[0] = 0;
  krr_pcg_opts o;
  krr_pcg_defaults(&o);
  if (opts) o = *opts;
  if (!X || !Y || !alpha) return fail(KRR_E_ARG, "krr_pcg_solve: null pointer");
  if (n < 1 || d < 1 || m < 1 || ldx < d || ldy < m || lda < m)
    return fail(KRR_E_ARG, "krr_pcg_solve: bad sizes or strides");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(KRR_E_ARG, "krr_pcg_solve: sigma must be > 0");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(KRR_E_ARG, "krr_pcg_solve: lambda must be > 0");
  if (!(o.tol > 0.0)) return fail(KRR_E_ARG, "krr_pcg_solve: tol must be > 0");
  if (o.max_iter < 1) return fail(KRR_E_ARG, "krr_pcg_solve: max_iter must be >= 1");
  if (!prec_ok(o.prec)) return fail(KRR_E_ARG, "krr_pcg_solve: unknown precision %d", o.prec);
  if (o.prec == KRR_PREC_BF16X3 && kp_for(d) > 256)
    return fail(KRR_E_ARG, "krr_pcg_solve: BF16X3 supports d <= 254 (d=%lld)", (long long)d);
  if (o.use_precond) {
    if (!Ut || s < 1 || s >= n || ldu < s)
      return fail(KRR_E_ARG, "krr_pcg_solve: preconditioner needs Ut with 1 <= s < n, ldu >= s");
  } else {
    s = 0;
  }
  if (o.check_every < 1) o.check_every = 1;
  const double lambda_p = o.lambda_p > 0.0 ? o.lambda_p : lambda;
  const size_t need = krr_workspace_bytes(KRR_OP_PCG_SOLVE, n, n, d, s, m, o.prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  PCGLayout L;
  layout_pcg(bb, L, n, d, s, m, o.prec);
  hipStream_t st = (hipStream_t)stream;
  const bool mixed = o.prec != KRR_PREC_FP64;
  CHECK_HIP(prepare_points(L.mm, X, ldx, nullptr, 0, sigma, st));
  if (mixed && (o.true_residual || o.refine > 0))
    CHECK_HIP(prepare_points(L.mm64, X, ldx, nullptr, 0, sigma, st));

  MMTimer timer;
  CHECK_HIP(timer.init());
  SolveArgs a{&L, n, m, s, ldu, Ut, lambda, lambda_p, o.tol, o.use_precond, o.max_iter,
              o.check_every, mixed, &timer};
  std::vector<double> hist;
  int iters = 0;
  if (!o.warm_start) CHECK_HIP(fill2d_zero(alpha, lda, n, m, st));
  CHECK_ST(pcg_core(a, Y, ldy, alpha, lda, o.warm_start != 0, &iters, &hist, st));
  int total_iters = iters;
  std::vector<int> h_broken(m);
  std::vector<double> h_rnorm(m), h_ynorm(m);
  auto fetch = [&]() -> krr_status {
    CHECK_HIP(hipMemcpyAsync(h_broken.data(), L.broken, sizeof(int) * m, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipMemcpyAsync(h_rnorm.data(), L.rnorm, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipMemcpyAsync(h_ynorm.data(), L.ynorm, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    CHECK_HIP(hipStreamSynchronize(st));
    return KRR_OK;
  };
  CHECK_ST(fetch());
  std::vector<int> broken0 = h_broken;
  std::vector<double> rel_rec(m), rel_true;
  for (int64_t c = 0; c < m; ++c) rel_rec[c] = h_ynorm[c] > 0 ? h_rnorm[c] / h_ynorm[c] : h_rnorm[c];
  int refine_steps = 0;
  if (o.true_residual || o.refine > 0) {
    CHECK_ST(true_residual(L, a, Y, ldy, alpha, lda, rel_true, st));
    while (refine_steps < o.refine) {
      double worst = 0.0;
      for (double v : rel_true) worst = std::max(worst, v);
      if (!(worst > o.tol)) break;
      // correction: A delta = R, R = Y - A alpha (in L.rhs); inner tolerance relative to R
      ++refine_steps;
      SolveArgs ai = a;
      ai.tol = std::max(0.5 * o.tol / worst, 1e-14);
      CHECK_HIP(copy2d(L.rhs, m, L.delta, m, n, m, st));  // keep R
      CHECK_HIP(fill_f64(L.ax, n * m, 0.0, st));
      // solve into L.ax (zero start), rhs = R (held in L.delta while L.rhs is reused)
      int it2 = 0;
      CHECK_ST(pcg_core(ai, L.delta, m, L.ax, m, false, &it2, &hist, st));
      total_iters += it2;
      CHECK_HIP(add2d(L.ax, m, alpha, lda, n, m, st));
      CHECK_ST(true_residual(L, a, Y, ldy, alpha, lda, rel_true, st));
    }
  }
  CHECK_HIP(timer.harvest());
  int conv = 0, brk = 0;
  for (int64_t c = 0; c < m; ++c) {
    if (broken0[c]) ++brk;
    if (!broken0[c] && rel_rec[c] <= o.tol) ++conv;
  }
  if (rep) {
    rep->iters = total_iters;
    rep->converged_cols = conv;
    rep->breakdown_cols = brk;
    rep->refine_steps = refine_steps;
    if (rep->relres_rec) for (int64_t c = 0; c < m; ++c) rep->relres_rec[c] = rel_rec[c];
    if (rep->relres_true)
      for (int64_t c = 0; c < m; ++c) rep->relres_true[c] = rel_true.empty() ? NAN : rel_true[c];
    int hl = 0;
    if (rep->history && rep->history_cap > 0)
      for (; hl < rep->history_cap && hl < (int)hist.size(); ++hl) rep->history[hl] = hist[hl];
    rep->history_len = hl;
    rep->matmat_calls = timer.calls;
    rep->matmat_ms = timer.ms;
  }
  if (brk > 0) return fail(KRR_E_BREAKDOWN, "krr_pcg_solve: %d column(s) broke down", brk);
  bool ok;
  if (refine_steps > 0) {
    ok = true;
    for (double v : rel_true) ok = ok && v <= o.tol;
  } else {
    ok = conv == m;
  }
  if (!ok) return fail(KRR_E_NO_CONV, "krr_pcg_solve: not converged after %d iterations", total_iters);
  return KRR_OK;
}

// ------------------------------------------------------------------------ grad
krr_status krr_grad(const float* X, int64_t n, int64_t d, int64_t ldx, double sigma,
                    const double* alpha, const double* abar, int64_t m, int64_t ld,
                    double* dL_dsigma, double* dL_dlambda, int32_t prec, void* ws, size_t ws_bytes,
                    void* stream) {
  g_err[0] = 0;
  if (!X || !alpha || !abar || !dL_dsigma || !dL_dlambda) return fail(KRR_E_ARG, "krr_grad: null pointer");
  if (n < 1 || d < 1 || m < 1 || ldx < d || ld < m) return fail(KRR_E_ARG, "krr_grad: bad sizes");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(KRR_E_ARG, "krr_grad: sigma must be > 0");
  if (!prec_ok(prec)) return fail(KRR_E_ARG, "krr_grad: unknown precision %d", prec);
  if (prec == KRR_PREC_BF16X3 && kp_for(d) > 256)
    return fail(KRR_E_ARG, "krr_grad: BF16X3 supports d <= 254 (d=%lld)", (long long)d);
  const size_t need = krr_workspace_bytes(KRR_OP_GRAD, n, n, d, 0, m, prec);
  CHECK_ST(check_ws(ws, ws_bytes, need));
  Bump bb(ws);
  GradLayout L;
  layout_grad(bb, L, n, d, m, prec);
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(prepare_points(L.mm, X, ldx, nullptr, 0, sigma, st));
  // W = (dK/dsigma) alpha
  if (prec == KRR_PREC_FP64) {
    CHECK_HIP(run_matmat(L.mm, nullptr, alpha, ld, true, st));
  } else {
    CHECK_HIP(vec_to_f32(alpha, n, m, ld, round_up(n, ROW_PAD), m, L.af, st));
    CHECK_HIP(run_matmat(L.mm, L.af, nullptr, m, true, st));
  }
  CHECK_HIP(matmat_finalize<double>(L.mm.part, L.mm.part_stride, L.mm.nsplit, n, m, m, 0.0, alpha,
                                    ld, L.w, m, st));
  CHECK_HIP(dot_partial<double, double>(abar, ld, L.w, m, n, m, L.part, NBLK, st));
  CHECK_HIP(dot_partial<double, double>(abar, ld, alpha, ld, n, m, L.part + NBLK * m, NBLK, st));
  std::vector<double> h(2 * NBLK * m);
  CHECK_HIP(hipMemcpyAsync(h.data(), L.part, sizeof(double) * 2 * NBLK * m, hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  double s1 = 0.0, s2 = 0.0;
  for (int64_t e = 0; e < NBLK * m; ++e) { s1 += h[e]; s2 += h[NBLK * m + e]; }
  *dL_dsigma = -s1;
  *dL_dlambda = -s2;
  return KRR_OK;
}

}  // extern "C"
