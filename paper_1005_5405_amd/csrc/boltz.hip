// boltz.hip -- host side of libboltz: problem validation, velocity-grid and
// sampling tables, context memory, and the C ABI declared in include/boltz.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "boltz.h"
#include "adjoint.hpp"
#include "kernels.hpp"
#include "sequential.hpp"

using namespace boltz;

namespace {

constexpr double kInvSqrtPi = 0.56418958354775628694807945156077;
constexpr double kTwoPi = 6.28318530717958647692528676655901;

thread_local std::string g_create_error;

}  // namespace

struct boltz_ctx {
  boltz_problem p{};
  int n[3]{};
  double a[3]{}, dvel[3]{}, inv_cell[3]{};
  std::vector<double> v[3], om[3], edge[3];
  std::vector<uint64_t> T[3];
  std::vector<double> pphi[3], punif[3];
  double dx = 0, dy = 0, dt = 0, K = 0, W = 0, qfac = 0;
  int nv = 0;
  int64_t ncells = 0;
  int device = 0;
  // spatial cell widths (Sec. 5.1 stretching, else 1/n) and whether stretched
  std::vector<double> wx, wy;
  bool sstretched = false;
  // device memory (one allocation)
  void* dmem = nullptr;
  size_t dbytes = 0;
  Params P{};
  // collide launch: block size, accumulator kind, dynamic LDS and persistent
  // grid of the fused-sampler [0] and shared-table [1] variants
  int collide_block[2] = {256, 256};
  int collide_mode = ACC_FIXED;  // accumulation of the increments (ACC_*)
  int batch_mode = ACC_FIXED;    // ... in batches (no ACC_HYBRID or ACC_PART there)
  int hyb_lo[2] = {0, 0}, hyb_n[2] = {0, 0};  // ACC_HYBRID / ACC_PART inner nodes per variant
  size_t collide_lds[2] = {0, 0};
  int64_t collide_grid[2] = {0, 0};
  int64_t ngroups = 0;          // sample groups (shared-sample mode)
  // wall state the ratio tables Phi_w / Phi0 were last built for
  WallArgs ratio_walls{};
  std::vector<double> ratio_taub;   // bottom-face temperatures of that state
  bool ratio_valid = false;
  // adjoint: collide-adjoint launch (block, dynamic LDS, grid) of the two
  // variants, and the scratch of BOLTZ_WITH_ADJOINT
  bool adj_supported = false;
  int adj_block = 256;
  bool adj_fixed[2] = {false, false};
  size_t adj_lds[2] = {0, 0};
  int64_t adj_grid[2] = {0, 0};
  float* adj_hs = nullptr;      // post-stream state recomputed by boltz_step_adjoint
  double* adj_lam = nullptr;    // FP64 adjoint of an intermediate state
  double* lnw = nullptr;        // adjoint of every face density
  double* gpart = nullptr;      // per-face wall-parameter partials [nfaces][2]
  uint2* tidx = nullptr;        // ngroups * n_pairs pair indices (G != 1)
  float4* tcoef = nullptr;      // ngroups * n_pairs pair coefficients
  uint2* sidx = nullptr;        // the sampler's output (ACC_SPLIT: sorted into tidx, tcoef)
  float4* scoef = nullptr;
  unsigned char* scratch = nullptr;  // this device's copy of the static record scratch
  // in-place sequential collision (BOLTZ_SEQUENTIAL_UPDATE): level of every
  // shared record, node velocities and weights of the three axes (FP64),
  // dynamic LDS
  bool seq = false;
  unsigned char* sched = nullptr;  // SeqSched of every sample group, or the levels (groups schedule)
  int seq_sched = 1;               // 1: steps of up to 64 records of one level; 0: groups of 64
  double* vom = nullptr;
  size_t seq_lds = 0;
  int collide_per_cu[2] = {0, 0};  // resident workgroups per CU of the two collide variants
  std::string err;
};

// Record scratch of boltz_collide_noalloc (see include/boltz.h): the shared
// pair records of one step, which that entry point keeps here instead of in
// the context.  One copy per device, held until the process ends; host code
// uses the address hipGetSymbolAddress returns for the current device (kept in
// every context created on it), never the array's name.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Where a collision reads its shared records: tidx, tcoef (what the kernel
// reads) and sidx, scoef (what the sampler writes; the same arrays unless
// the split layout sorts them).
struct RecordTables {
  uint2* tidx;
  float4* tcoef;
  uint2* sidx;
  float4* scoef;
  unsigned char* sched = nullptr;  // sequential collision: the step schedule (SeqSched)
};

namespace {

int fail(boltz_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return code;
}

int hip_fail(boltz_ctx* c, hipError_t e, const char* what) {
  return fail(c, BOLTZ_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WallArgs make_walls(const boltz_walls* w) {
  WallArgs a{};
  a.lid_u = w ? w->lid_u : 0.0;
  const double t[4] = {w ? w->tau_left : 1.0, w ? w->tau_right : 1.0, w ? w->tau_bottom : 1.0,
                       w ? w->tau_top : 1.0};
  for (int k = 0; k < 4; ++k) {
    a.tau[k] = t[k];
    a.tfac[k] = std::pow(t[k], -1.5);
  }
  return a;
}

bool walls_ok(const boltz_walls* w, int nx) {
  if (!(w && w->tau_left > 0 && w->tau_right > 0 && w->tau_bottom > 0 && w->tau_top > 0 &&
        std::isfinite(w->lid_u) && std::isfinite(w->tau_left) && std::isfinite(w->tau_right) &&
        std::isfinite(w->tau_bottom) && std::isfinite(w->tau_top)))
    return false;
  if (w->tau_bottom_x)
    for (int i = 0; i < nx; ++i)
      if (!(w->tau_bottom_x[i] > 0) || !std::isfinite(w->tau_bottom_x[i])) return false;
  return true;
}

// temperatures of the bottom faces of a wall state
std::vector<double> bottom_taus(const boltz_walls* w, int nx) {
  std::vector<double> t(nx, w ? w->tau_bottom : 1.0);
  if (w && w->tau_bottom_x)
    for (int i = 0; i < nx; ++i) t[i] = w->tau_bottom_x[i];
  return t;
}

constexpr size_t kLdsBytes = 160 * 1024;

// static LDS of the collide kernel (block reduction scratch and flags) per
// block size
size_t collide_static_lds(int block) { return 20 * (size_t)(block / 64) * sizeof(double) + 96; }

// ACC_HYBRID for grids whose 64-bit layout does not fit: the most x-slabs
// (centred; at least half of them) whose 64-bit accumulators fit next to the
// h^s tile, the FP32 accumulators of the other slabs and the tables, with
// 1024 threads.  lo, nin: first inner node and inner node count.
bool pick_hybrid(const int (&n)[3], int ns, bool sampler, int& lo, int& nin) {
  const int slab = n[1] * n[2], nv = n[0] * slab;
  for (int S = n[0]; S >= (n[0] + 1) / 2 && S >= 1; --S) {
    const int nn = S * slab;
    if (CollideLDS::hyb_bytes(nv, nn, ns, sampler) + collide_static_lds(1024) <= kLdsBytes) {
      lo = ((n[0] - S) / 2) * slab;
      nin = nn;
      return true;
    }
  }
  return false;
}

// ACC_PART for grids whose 64-bit layout does not fit: the most x-slabs
// (centred; at least half of them) whose FP32 h^s tile fits after the
// 64-bit accumulators of every node and the tables, with 1024 threads.
bool pick_part(const int (&n)[3], int ns, bool sampler, int& lo, int& nin) {
  const int slab = n[1] * n[2], nv = n[0] * slab;
  for (int S = n[0]; S >= (n[0] + 1) / 2 && S >= 1; --S) {
    const int nn = S * slab;
    if (CollideLDS::part_bytes(nv, nn, ns, sampler) + collide_static_lds(1024) <= kLdsBytes) {
      lo = ((n[0] - S) / 2) * slab;
      nin = nn;
      return true;
    }
  }
  return false;
}

// Accumulation mode and block sizes of the collide kernel: 64-bit
// fixed-point accumulators for every node when they fit next to the h tile
// and tables, else for half of the nodes per pass, else FP32; the block size
// gives about 1024 resident threads per CU.  block[0]: pairs drawn in the
// kernel; block[1]: pairs read from the shared table (1024 threads: 289 us
// per collision on the 64x64 cavity against 311 us with 512).  The split
// mode keeps 8192 / block nodes per thread in registers between its
// passes, and uses 512 threads.
bool pick_collide(int nv, int ns, int& mode, int (&blocks)[2]) {
  int block = 256;
  if (CollideLDS::bytes(nv, ns, ACC_FIXED, true) + collide_static_lds(1024) <= kLdsBytes) mode = ACC_FIXED;
  else if (CollideLDS::bytes(nv, ns, ACC_SPLIT, true) + collide_static_lds(512) <= kLdsBytes &&
           CollideLDS::half(nv) <= 8192)
    mode = ACC_SPLIT;
  else mode = ACC_CAS;
  const size_t dyn = CollideLDS::bytes(nv, ns, mode, true);
  if (dyn + collide_static_lds(1024) > kLdsBytes && mode != ACC_SPLIT) return false;
  if (4 * (dyn + collide_static_lds(256)) <= kLdsBytes) block = 256;
  else if (2 * (dyn + collide_static_lds(512)) <= kLdsBytes || mode == ACC_SPLIT) block = 512;
  else block = 1024;
  blocks[0] = blocks[1] = block;
  // tuning override: BOLTZ_COLLIDE_BLOCK = 256 | 512 | 1024 (both variants)
  if (const char* e = std::getenv("BOLTZ_COLLIDE_BLOCK")) {
    const int b = std::atoi(e);
    if ((b == 256 || b == 512 || b == 1024) && dyn + collide_static_lds(b) <= kLdsBytes) blocks[0] = blocks[1] = b;
  }
  return true;
}

// Block size of the collide adjoint (at least the FP64-sum layout, the
// forward's fixed-point layout plus a y . psi table, must fit in LDS): 256
// threads when four workgroups fit per CU, else 512.  fixed[t]: the
// fixed-point adjoint sums (one more FP32 array) fit as well, for the
// drawn-pair [0] and shared-table [1] variants.  false when nothing fits.
bool pick_adjoint(int nv, int ns, int& block, bool (&fixed)[2]) {
  const size_t dyn = collide_adj_lds(nv, ns, true, false);
  if (dyn + collide_adj_static_lds(512) > kLdsBytes) return false;
  block = (4 * (dyn + collide_adj_static_lds(256)) <= kLdsBytes) ? 256 : 512;
  for (int t = 0; t < 2; ++t)
    fixed[t] = collide_adj_lds(nv, ns, t == 0, true) + collide_adj_static_lds(block) <= kLdsBytes;
  return true;
}

const void* collide_adj_fn(int block, bool table, bool fixed) {
#define BOLTZ_ADJ_FN(B)                                                                                   \
  if (block == B)                                                                                         \
    return table ? (fixed ? (const void*)collide_adj_kernel<B, true, true> : (const void*)collide_adj_kernel<B, true, false>) \
                 : (fixed ? (const void*)collide_adj_kernel<B, false, true> : (const void*)collide_adj_kernel<B, false, false>);
  BOLTZ_ADJ_FN(256)
  BOLTZ_ADJ_FN(512)
#undef BOLTZ_ADJ_FN
  return nullptr;
}

// table: shared records; else pairs drawn in the kernel by the node law or,
// with cont, from the continuous Maxwellian
const void* collide_fn(int block, bool table, int mode, bool cont = false) {
#define BOLTZ_COLLIDE_FN(B, M)                                                                                 \
  if (block == B && mode == M)                                                                                 \
    return table ? (const void*)collide_kernel<B, true, M>                                                     \
                 : (cont ? (const void*)collide_kernel<B, false, M, 2> : (const void*)collide_kernel<B, false, M, 1>);
  BOLTZ_COLLIDE_FN(256, ACC_FIXED)
  BOLTZ_COLLIDE_FN(512, ACC_FIXED)
  BOLTZ_COLLIDE_FN(1024, ACC_FIXED)
  BOLTZ_COLLIDE_FN(256, ACC_SPLIT)
  BOLTZ_COLLIDE_FN(512, ACC_SPLIT)
  BOLTZ_COLLIDE_FN(1024, ACC_SPLIT)
  BOLTZ_COLLIDE_FN(256, ACC_CAS)
  BOLTZ_COLLIDE_FN(512, ACC_CAS)
  BOLTZ_COLLIDE_FN(1024, ACC_CAS)
  BOLTZ_COLLIDE_FN(1024, ACC_HYBRID)
  BOLTZ_COLLIDE_FN(1024, ACC_PART)
#undef BOLTZ_COLLIDE_FN
  return nullptr;
}

}  // namespace

extern "C" {

const char* boltz_last_error(const boltz_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

void boltz_destroy(boltz_ctx* ctx) {
  if (!ctx) return;
  if (ctx->dmem) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->dmem);
    (void)hipSetDevice(cur);
  }
  delete ctx;
}

int boltz_create(const boltz_problem* p, boltz_ctx** out) {
  if (!p || !out) return fail(nullptr, BOLTZ_EINVAL, "boltz_create: null argument");
  *out = nullptr;
  const int min_cells = (p->bc == BOLTZ_BC_CAVITY) ? 2 : 1;
  if (p->nx < min_cells || p->ny < min_cells || p->nx > 100000 || p->ny > 100000)
    return fail(nullptr, BOLTZ_EINVAL, "boltz_create: nx, ny out of range (cavity needs >= 2 per axis)");
  for (int k = 0; k < 3; ++k)
    if (p->nv[k] < 1 || p->nv[k] > kMaxAxis || !(p->vmax[k] > 0.0) || !std::isfinite(p->vmax[k]))
      return fail(nullptr, BOLTZ_EINVAL, "boltz_create: velocity grid out of range (1 <= nv <= 255, vmax > 0)");
  if (!(p->delta > 0.0) || !(p->eps > 0.0) || (p->order != 1 && p->order != 2) ||
      (p->bc != BOLTZ_BC_CAVITY && p->bc != BOLTZ_BC_PERIODIC) || p->n_pairs < 0 ||
      p->n_pairs >= ((int64_t)1 << 31) || p->sample_group < 0 || p->mix16 > 16 ||
      (!(p->dt > 0.0) && !(p->cfl > 0.0)) ||
      (p->flags & ~(uint32_t)(BOLTZ_ALLOW_UNSTABLE | BOLTZ_WITH_ADJOINT | BOLTZ_CONTINUOUS_PAIRS |
                              BOLTZ_SEQUENTIAL_UPDATE)))
    return fail(nullptr, BOLTZ_EINVAL, "boltz_create: invalid scalar parameter");
  const bool seq = (p->flags & BOLTZ_SEQUENTIAL_UPDATE) != 0;
  if (seq && p->sample_group == 1)
    return fail(nullptr, BOLTZ_EINVAL,
                "boltz_create: the sequential update needs shared samples (sample_group 0 or >= 2): its "
                "record order is worked out once per sample group and step");
  if (seq && (p->flags & BOLTZ_WITH_ADJOINT))
    return fail(nullptr, BOLTZ_EINVAL, "boltz_create: the adjoint follows the Jacobi collision only");
  const bool sx_str = p->rx != 0.0 && p->rx != 1.0, sy_str = p->ry != 0.0 && p->ry != 1.0;
  if ((sx_str && !(p->rx > 0.0 && p->rx < 1.0)) || (sy_str && !(p->ry > 0.0 && p->ry < 1.0)) ||
      ((sx_str || sy_str) && p->order != 1))
    return fail(nullptr, BOLTZ_EINVAL,
                "boltz_create: stretched spatial cells need 0 < rx, ry < 1 and first-order streaming");
  if ((sx_str || sy_str) && (p->flags & BOLTZ_WITH_ADJOINT))
    return fail(nullptr, BOLTZ_EINVAL, "boltz_create: the adjoint follows uniform spatial cells only");
  if (seq && (int64_t)p->nx * p->ny > 0x7fffffffLL)
    return fail(nullptr, BOLTZ_EINVAL, "boltz_create: the sequential collision takes at most 2^31 - 1 cells");
  const bool stretched = p->rv != 0.0 && p->rv != 1.0;
  if (stretched && (!(p->rv > 0.0 && p->rv < 1.0) || (p->nv[0] & 1) || (p->nv[1] & 1) || (p->nv[2] & 1)))
    return fail(nullptr, BOLTZ_EINVAL,
                "boltz_create: a stretched velocity grid needs 0 < rv < 1 and an even cell count per axis");
  const int64_t nvt = (int64_t)p->nv[0] * p->nv[1] * p->nv[2];
  const int nsum = p->nv[0] + p->nv[1] + p->nv[2];
  int cmode = ACC_FIXED;
  int cblock[2] = {256, 256};
  if (nvt > (1 << 20) || (!pick_collide((int)nvt, nsum, cmode, cblock) && !seq))
    return fail(nullptr, BOLTZ_EUNSUPPORTED,
                "boltz_create: the per-cell h and increment tiles of this velocity grid exceed the 160 KB LDS");
  // a single problem whose grid is too large for the 64-bit layout collides
  // in one pass with ACC_PART, else ACC_HYBRID; batches keep the classic
  // layouts.  The sequential collision has a kernel of its own (the Jacobi
  // set-up below is skipped).
  if (seq) {
    cmode = ACC_FIXED;
    cblock[0] = cblock[1] = 256;
  }
  const int bmode = cmode;
  int hlo[2] = {0, 0}, hn[2] = {0, 0};
  if (cmode != ACC_FIXED && nvt <= 65535) {
    const char* lay = std::getenv("BOLTZ_COLLIDE_LAYOUT");
    const bool no_part = lay && std::strcmp(lay, "hybrid") == 0;
    if (!no_part && pick_part(p->nv, nsum, true, hlo[0], hn[0]) && pick_part(p->nv, nsum, false, hlo[1], hn[1])) {
      cmode = ACC_PART;
      cblock[0] = cblock[1] = 1024;
    } else if (pick_hybrid(p->nv, nsum, true, hlo[0], hn[0]) && pick_hybrid(p->nv, nsum, false, hlo[1], hn[1])) {
      cmode = ACC_HYBRID;
      cblock[0] = cblock[1] = 1024;
    }
  }
  if ((int64_t)p->nx * p->ny * nvt >= ((int64_t)1 << 40))
    return fail(nullptr, BOLTZ_EINVAL, "boltz_create: phase-space grid too large");
  const int64_t ncells_ = (int64_t)p->nx * p->ny;
  const int64_t ngroups = (p->sample_group == 1) ? 0
                          : (p->sample_group == 0 ? 1 : (ncells_ + p->sample_group - 1) / p->sample_group);
  if (ngroups > 65535 || nvt > 65535)
    return fail(nullptr, BOLTZ_EINVAL,
                "boltz_create: shared-sample mode needs at most 65535 groups and 65535 velocity nodes");
  if (seq && SeqLDS::bytes((int)nvt, nsum) > kLdsBytes)
    return fail(nullptr, BOLTZ_EUNSUPPORTED,
                "boltz_create: the h tile of the sequential collision exceeds the 160 KB LDS");

  boltz_ctx* c = new (std::nothrow) boltz_ctx;
  if (!c) return fail(nullptr, BOLTZ_ENOMEM, "boltz_create: out of host memory");
  c->p = *p;
  c->nv = (int)nvt;
  c->ncells = (int64_t)p->nx * p->ny;
  // Sec. 3: uniform velocity cells on [-a, a], node at the cell centre;
  // omega = dv exp(-v^2)/sqrt(pi) is the per-axis midpoint weight of Phi0.
  for (int k = 0; k < 3; ++k) {
    const int n = p->nv[k];
    const double a = p->vmax[k];
    c->n[k] = n;
    c->a[k] = a;
    c->dvel[k] = (2.0 * a) / n;
    c->inv_cell[k] = (double)n / (2.0 * a);
    c->v[k].resize(n);
    c->om[k].resize(n);
    c->edge[k].resize(n + 1);
    c->T[k].assign(n, 0);
    double osum = 0.0;
    if (!stretched) {
      for (int i = 0; i < n; ++i) {
        const double vi = ((double)(2 * i + 1 - n) * a) / n;
        c->v[k][i] = vi;
        c->om[k][i] = (c->dvel[k] * std::exp(-(vi * vi))) * kInvSqrtPi;
        osum += c->om[k][i];
      }
      for (int i = 0; i <= n; ++i) c->edge[k][i] = -a + i * c->dvel[k];
    } else {
      // Sec. 5.1: the i-th cell from the origin on each half axis is
      // w0 rv^-i long (the smallest at the origin, lengths adding up to a,
      // outermost edge a exactly); nodes at the cell centres, the negative
      // half the mirror image of the positive one
      const int m = n / 2;
      double sum = 0.0, t = 1.0;
      for (int i = 0; i < m; ++i) {
        sum += t;
        t /= p->rv;
      }
      const double w0 = a / sum;
      std::vector<double> E(m + 1, 0.0);
      t = 1.0;
      for (int i = 0; i < m; ++i) {
        E[i + 1] = E[i] + w0 * t;
        t /= p->rv;
      }
      E[m] = a;
      for (int i = 0; i <= m; ++i) {
        c->edge[k][m + i] = E[i];
        c->edge[k][m - i] = -E[i];
      }
      for (int i = 0; i < m; ++i) {
        const double vi = 0.5 * (E[i] + E[i + 1]);
        c->v[k][m + i] = vi;
        c->v[k][m - 1 - i] = -vi;
      }
      for (int i = 0; i < n; ++i) {
        const double vi = c->v[k][i];
        c->om[k][i] = ((c->edge[k][i + 1] - c->edge[k][i]) * std::exp(-(vi * vi))) * kInvSqrtPi;
        osum += c->om[k][i];
      }
    }
    // node law of one axis on a 12-bit field f: node i for f in
    // [T_i, T_{i+1}), T_i = round(2^12 sum_{l<i} omega_l / sum omega)
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      if (i > 0) c->T[k][i] = (uint64_t)std::nearbyint(std::ldexp(s / osum, kFieldBits));
      s += c->om[k][i];
    }
    // realised probabilities: Maxwellian law (T_{i+1} - T_i) 2^-12; uniform
    // law floor(f n / 2^12): #{f : floor(f n 2^-12) = i} 2^-12
    c->pphi[k].resize(n);
    c->punif[k].resize(n);
    for (int i = 0; i < n; ++i) {
      const uint64_t hi = (i + 1 < n) ? c->T[k][i + 1] : ((uint64_t)1 << kFieldBits);
      c->pphi[k][i] = std::ldexp((double)(hi - c->T[k][i]), -kFieldBits);
      const uint64_t lo_u = (((uint64_t)i << kFieldBits) + (uint64_t)n - 1) / (uint64_t)n;
      const uint64_t hi_u = (((uint64_t)(i + 1) << kFieldBits) + (uint64_t)n - 1) / (uint64_t)n;
      c->punif[k][i] = std::ldexp((double)(hi_u - lo_u), -kFieldBits);
    }
  }
  // Eq. coll8Dim as an importance-sampling estimate is unbiased only if
  // every node the integrand reaches can be drawn: the Maxwellian law on
  // 12-bit fields gives probability zero to the far-tail nodes of wide grids,
  // so without the uniform component (mix16 = 0) it is refused there (the
  // continuous sampler does not use the node law).
  if (p->mix16 == 0 && !(p->flags & BOLTZ_CONTINUOUS_PAIRS))
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < c->n[k]; ++i)
        if (!(c->pphi[k][i] > 0.0)) {
          delete c;
          return fail(nullptr, BOLTZ_EINVAL,
                      "boltz_create: mix16 = 0: the Maxwellian node law gives probability zero to tail nodes "
                      "of this velocity grid (biased estimate); use mix16 > 0");
        }
  {
    // W = (Om_x Om_y) Om_z, the discrete mass of Phi0
    double Om[3];
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int i = 0; i < c->n[k]; ++i) s += c->om[k][i];
      Om[k] = s;
    }
    c->W = (Om[0] * Om[1]) * Om[2];
  }
  c->dx = 1.0 / p->nx;
  c->dy = 1.0 / p->ny;
  // Sec. 5.1: spatial cell lengths in geometric progression, the cell d
  // cells from the nearer side wall w0 rx^-d long (x), the cell d cells
  // below the lid w0 ry^-d (y), adding up to the cavity side 1
  c->sstretched = sx_str || sy_str;
  c->wx.assign(p->nx, 1.0);
  c->wy.assign(p->ny, 1.0);
  {
    double sum = 0.0;
    for (int i = 0; i < p->nx; ++i) {
      const int d = std::min(i, p->nx - 1 - i);
      if (sx_str) c->wx[i] = std::pow(p->rx, -d);
      sum += c->wx[i];
    }
    for (double& w : c->wx) w /= sum;
    sum = 0.0;
    for (int i = 0; i < p->ny; ++i) {
      if (sy_str) c->wy[i] = std::pow(p->ry, -(p->ny - 1 - i));
      sum += c->wy[i];
    }
    for (double& w : c->wy) w /= sum;
  }
  const double mwx = c->sstretched ? *std::min_element(c->wx.begin(), c->wx.end()) : c->dx;
  const double mwy = c->sstretched ? *std::min_element(c->wy.begin(), c->wy.end()) : c->dy;
  const double vmx = std::fabs(c->v[0][0]), vmy = std::fabs(c->v[1][0]);
  if (p->dt > 0.0) {
    c->dt = p->dt;
  } else {
    // the largest Courant number over nodes, cells and axes equals cfl
    const double rx = vmx / mwx, ry = vmy / mwy;
    c->dt = p->cfl / (rx > ry ? rx : ry);
  }
  const double cx = vmx * c->dt / mwx, cy = vmy * c->dt / mwy;
  const bool stable = (p->order == 1) ? (cx + cy <= 1.0 + 1e-12) : (cx <= 1.0 + 1e-12 && cy <= 1.0 + 1e-12);
  if (!stable && !(p->flags & BOLTZ_ALLOW_UNSTABLE)) {
    delete c;
    return fail(nullptr, BOLTZ_EINVAL, "boltz_create: time step violates the Courant limit of the streaming scheme");
  }
  // K = pi n0 sigma^2 from lambda0 = mu0/p0 sqrt(2RT0) and the hard-sphere
  // viscosity with the Chapman-Cowling factor 1.016034 (Sec. 5.1 scales).
  c->K = 0.3125 * std::sqrt(kTwoPi) * 1.016034 * p->delta;
  c->qfac = (p->n_pairs > 0) ? (c->dt * c->K) / (double)p->n_pairs : 0.0;

  // ---- host images of the device tables
  std::vector<double> vtab(3 * kMaxAxis, 0.0), omtab(3 * kMaxAxis, 0.0), rwtab(3 * kMaxAxis, 0.0);
  std::vector<double> edgetab(3 * (kMaxAxis + 1), 0.0);
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i <= c->n[k]; ++i) edgetab[k * (kMaxAxis + 1) + i] = c->edge[k][i];
  std::vector<float4> nqtab(3 * kMaxAxis, make_float4(0.f, 0.f, 0.f, 0.f));
  std::vector<uint8_t> icdf(3 * kFieldSize, 0);
  std::vector<float> cour(2 * kMaxAxis, 0.f), cour2(2 * kMaxAxis, 0.f);
  // omega_z v_z^p (p = 0..4) per z node, eight doubles a node
  std::vector<double> zmom((size_t)8 * c->n[2], 0.0);
  for (int i = 0; i < c->n[2]; ++i) {
    const double z = c->v[2][i], z2 = z * z;
    const double pw[5] = {1.0, z, z2, z2 * z, z2 * z2};
    for (int q = 0; q < 5; ++q) zmom[(size_t)8 * i + q] = c->om[2][i] * pw[q];
  }
  for (int k = 0; k < 3; ++k) {
    const int n = c->n[k];
    for (int i = 0; i < n; ++i) {
      vtab[k * kMaxAxis + i] = c->v[k][i];
      omtab[k * kMaxAxis + i] = c->om[k][i];
      rwtab[k * kMaxAxis + i] = 1.0 / c->om[k][i];
      nqtab[k * kMaxAxis + i] =
          make_float4((float)c->om[k][i], (float)c->pphi[k][i], (float)c->punif[k][i], 0.f);
    }
    // direct inverse CDF of the Maxwellian law: icdf[f] = #{i >= 1 : T_i <= f}
    int idx = 0;
    for (int f = 0; f < kFieldSize; ++f) {
      while (idx + 1 < n && c->T[k][idx + 1] <= (uint64_t)f) ++idx;
      icdf[k * kFieldSize + f] = (uint8_t)idx;
    }
  }
  // M0 = sum_j w_j psi_k psi_l, psi = (1, v_x, v_y, v_z, |v|^2), packed k <= l
  std::vector<double> m0(16, 0.0);
  for (int ix = 0; ix < c->n[0]; ++ix)
    for (int iy = 0; iy < c->n[1]; ++iy)
      for (int iz = 0; iz < c->n[2]; ++iz) {
        const double vx = c->v[0][ix], vy = c->v[1][iy], vz = c->v[2][iz];
        const double w = (c->om[0][ix] * c->om[1][iy]) * c->om[2][iz];
        const double psi[5] = {1.0, vx, vy, vz, (vx * vx + vy * vy) + vz * vz};
        int t = 0;
        for (int k = 0; k < 5; ++k)
          for (int l = k; l < 5; ++l) m0[t++] += w * psi[k] * psi[l];
      }
  for (int k = 0; k < 2; ++k) {
    const double dl = k == 0 ? c->dx : c->dy;
    for (int i = 0; i < c->n[k]; ++i) {
      const double C = std::fabs(c->v[k][i]) * c->dt / dl;
      cour[k * kMaxAxis + i] = (float)C;
      cour2[k * kMaxAxis + i] = (float)(0.5 * C * (1.0 - C));
    }
  }
  // ---- device memory: tables + scratch in one allocation
  const int nfaces = 2 * (p->nx + p->ny);
  size_t off = 0;
  const size_t o_v = off; off = align256(off + vtab.size() * 8);
  const size_t o_edge = off; off = align256(off + edgetab.size() * 8);
  const size_t o_om = off; off = align256(off + omtab.size() * 8);
  const size_t o_rw = off; off = align256(off + rwtab.size() * 8);
  const size_t o_nq = off; off = align256(off + nqtab.size() * 16);
  const size_t o_icdf = off; off = align256(off + icdf.size());
  const size_t o_m0 = off; off = align256(off + m0.size() * 8);
  const size_t o_zmom = off; off = align256(off + zmom.size() * 8);
  const size_t o_cour = off; off = align256(off + cour.size() * 4);
  const size_t o_cour2 = off; off = align256(off + cour2.size() * 4);
  const size_t o_nw = off; off = align256(off + (size_t)nfaces * 8);
  const size_t o_ratio = off; off = align256(off + (size_t)4 * c->nv * 8);
  const size_t o_ratio_b = off; off = align256(off + (size_t)p->nx * c->nv * 8);
  const size_t o_tau_b = off; off = align256(off + (size_t)p->nx * 8);
  const size_t o_wconst_b = off; off = align256(off + (size_t)p->nx * 2 * 8);
  const size_t o_dpart = off; off = align256(off + (size_t)p->nx * 8);
  const size_t o_wconst = off; off = align256(off + 8 * 8);
  const size_t o_status = off; off = align256(off + 4);
  const size_t o_lnw = off; off = align256(off + (size_t)nfaces * 8);
  const size_t o_gpart = off; off = align256(off + (size_t)nfaces * 2 * 8);
  const size_t o_tidx = off; off = align256(off + (size_t)ngroups * (size_t)p->n_pairs * sizeof(uint2));
  const size_t o_tcoef = off; off = align256(off + (size_t)ngroups * (size_t)p->n_pairs * sizeof(float4));
  const size_t nsort = (bmode == ACC_SPLIT) ? (size_t)ngroups * (size_t)p->n_pairs : 0;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess || ncu < 1) ncu = 256;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu < 1) ncu = 256;
  }
  // ACC_HYBRID, ACC_PART: one global row per persistent workgroup (at most two per CU)
  const int64_t hyb_rows = (cmode == ACC_HYBRID || cmode == ACC_PART) ? 2 * (int64_t)ncu : 0;
  const size_t o_hyb = off; off = align256(off + (size_t)hyb_rows * (size_t)nvt * 4);
  const size_t o_sidx = off; off = align256(off + nsort * sizeof(uint2));
  const size_t o_scoef = off; off = align256(off + nsort * sizeof(float4));
  const bool with_adj = (p->flags & BOLTZ_WITH_ADJOINT) != 0;
  const size_t nodes = (size_t)c->ncells * (size_t)c->nv;
  const size_t o_adj_hs = off; off = align256(off + (with_adj ? nodes * 4 : 0));
  const size_t o_adj_lam = off; off = align256(off + (with_adj ? nodes * 8 : 0));
  const int64_t ngr_seq = (p->n_pairs + kSeqGroup - 1) / kSeqGroup;
  const size_t o_sched = off; off = align256(off + (seq ? SeqSched::bytes(ngr_seq, ngroups) : 0));
  std::vector<double> vom(2 * (size_t)nsum, 0.0);
  {
    size_t i = 0;
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < c->n[k]; ++j, ++i) {
        vom[i] = c->v[k][j];
        vom[nsum + i] = c->om[k][j];
      }
  }
  const size_t o_vom = off; off = align256(off + vom.size() * 8);
  // stretched spatial cells: x widths, 1 / x widths, 1 / y widths
  std::vector<double> swid;
  if (c->sstretched) {
    for (double w : c->wx) swid.push_back(w);
    for (double w : c->wx) swid.push_back(1.0 / w);
    for (double w : c->wy) swid.push_back(1.0 / w);
  }
  const size_t o_swid = off; off = align256(off + swid.size() * 8);
  (void)hipGetDevice(&c->device);
  hipError_t e = hipMalloc(&c->dmem, off);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, BOLTZ_ENOMEM, std::string("boltz_create: hipMalloc: ") + hipGetErrorString(e));
  }
  c->dbytes = off;
  unsigned char* base = static_cast<unsigned char*>(c->dmem);
  struct Cp { size_t o; const void* src; size_t n; } cps[] = {
      {o_v, vtab.data(), vtab.size() * 8}, {o_edge, edgetab.data(), edgetab.size() * 8},
      {o_om, omtab.data(), omtab.size() * 8},
      {o_rw, rwtab.data(), rwtab.size() * 8}, {o_nq, nqtab.data(), nqtab.size() * 16},
      {o_icdf, icdf.data(), icdf.size()}, {o_m0, m0.data(), m0.size() * 8},
      {o_zmom, zmom.data(), zmom.size() * 8},
      {o_cour, cour.data(), cour.size() * 4}, {o_cour2, cour2.data(), cour2.size() * 4},
      {o_vom, vom.data(), vom.size() * 8}, {o_swid, swid.data(), swid.size() * 8}};
  for (const Cp& cp : cps) {
    e = hipMemcpy(base + cp.o, cp.src, cp.n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      boltz_destroy(c);
      return fail(nullptr, BOLTZ_EHIP, std::string("boltz_create: hipMemcpy: ") + hipGetErrorString(e));
    }
  }
  e = hipMemset(base + o_nw, 0, o_status + 4 - o_nw);
  if (e == hipSuccess && hyb_rows) e = hipMemset(base + o_hyb, 0, (size_t)hyb_rows * (size_t)nvt * 4);
  if (e != hipSuccess) {
    boltz_destroy(c);
    return fail(nullptr, BOLTZ_EHIP, std::string("boltz_create: hipMemset: ") + hipGetErrorString(e));
  }
  Params& P = c->P;
  P.nx = p->nx;
  P.ny = p->ny;
  P.nv = c->nv;
  for (int k = 0; k < 3; ++k) {
    P.n[k] = c->n[k];
    P.a[k] = c->a[k];
    P.inv_cell[k] = c->inv_cell[k];
    // sign ranges of the (increasing) node velocities of axis k
    int neg = 0, pos = 0;
    for (int i = 0; i < c->n[k]; ++i) {
      if (c->v[k][i] < 0.0) neg = i + 1;
      if (c->v[k][i] <= 0.0) pos = i + 1;
    }
    P.vneg[k] = neg;
    P.vpos[k] = pos;
  }
  P.order = p->order;
  P.bc = p->bc;
  P.n_pairs = p->n_pairs;
  P.sample_group = p->sample_group;
  P.key0 = (uint32_t)p->seed;
  P.key1 = (uint32_t)(p->seed >> 32);
  P.cavity = p->cavity_id;
  P.mix16 = p->mix16;
  P.beta = p->mix16 / 16.0;
  P.dt = c->dt;
  P.dx = c->dx;
  P.dy = c->dy;
  P.eps = p->eps;
  P.inv_eps = 1.0 / p->eps;
  P.qfac = c->qfac;

  P.vtab = reinterpret_cast<const double*>(base + o_v);
  P.stretched = stretched ? 1 : 0;
  P.continuous = (p->flags & BOLTZ_CONTINUOUS_PAIRS) ? 1 : 0;
  P.wx = c->sstretched ? reinterpret_cast<const double*>(base + o_swid) : nullptr;
  P.inv_wx = c->sstretched ? P.wx + p->nx : nullptr;
  P.inv_wy = c->sstretched ? P.wx + 2 * p->nx : nullptr;
  P.edgetab = reinterpret_cast<const double*>(base + o_edge);
  P.omtab = reinterpret_cast<const double*>(base + o_om);
  P.rwtab = reinterpret_cast<const double*>(base + o_rw);
  P.nqtab = reinterpret_cast<const float4*>(base + o_nq);
  P.icdf = reinterpret_cast<const uint8_t*>(base + o_icdf);
  P.m0 = reinterpret_cast<const double*>(base + o_m0);
  P.zmom = reinterpret_cast<const double*>(base + o_zmom);
  P.cour = reinterpret_cast<const float*>(base + o_cour);
  P.cour2 = reinterpret_cast<const float*>(base + o_cour2);
  P.nw = reinterpret_cast<double*>(base + o_nw);
  P.ratio = reinterpret_cast<double*>(base + o_ratio);
  P.ratio_b = reinterpret_cast<double*>(base + o_ratio_b);
  P.tau_b = reinterpret_cast<const double*>(base + o_tau_b);
  P.wconst_b = reinterpret_cast<double*>(base + o_wconst_b);
  P.dpart = reinterpret_cast<double*>(base + o_dpart);
  P.wconst = reinterpret_cast<double*>(base + o_wconst);
  P.status = reinterpret_cast<uint32_t*>(base + o_status);
  P.hyb_lo = hlo[1];
  P.hyb_n = hn[1];
  P.hyb_ovf = hyb_rows ? reinterpret_cast<float*>(base + o_hyb) : nullptr;
  c->ngroups = ngroups;
  c->tidx = ngroups ? reinterpret_cast<uint2*>(base + o_tidx) : nullptr;
  c->tcoef = ngroups ? reinterpret_cast<float4*>(base + o_tcoef) : nullptr;
  c->sidx = nsort ? reinterpret_cast<uint2*>(base + o_sidx) : c->tidx;
  c->scoef = nsort ? reinterpret_cast<float4*>(base + o_scoef) : c->tcoef;
  c->lnw = reinterpret_cast<double*>(base + o_lnw);
  c->gpart = reinterpret_cast<double*>(base + o_gpart);
  c->adj_hs = with_adj ? reinterpret_cast<float*>(base + o_adj_hs) : nullptr;
  c->adj_lam = with_adj ? reinterpret_cast<double*>(base + o_adj_lam) : nullptr;
  c->seq = seq;
  c->sched = seq ? base + o_sched : nullptr;
  c->vom = reinterpret_cast<double*>(base + o_vom);
  c->seq_lds = SeqLDS::bytes(c->nv, nsum);
  c->collide_block[0] = cblock[0];
  c->collide_block[1] = cblock[1];
  c->collide_mode = cmode;
  c->batch_mode = bmode;
  for (int t = 0; t < 2; ++t) {
    c->hyb_lo[t] = hlo[t];
    c->hyb_n[t] = hn[t];
  }
  // this device's address of the static record scratch (boltz_collide_noalloc)
  {
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) == hipSuccess) c->scratch = static_cast<unsigned char*>(sp);
    else (void)hipGetLastError();
  }
  hipError_t ea = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  for (int t = 0; t < 2 && ea == hipSuccess && !seq; ++t) {
    const void* fn = collide_fn(cblock[t], t == 1, cmode, (p->flags & BOLTZ_CONTINUOUS_PAIRS) != 0);
    c->collide_lds[t] = cmode == ACC_HYBRID ? CollideLDS::hyb_bytes(c->nv, hn[t], nsum, t == 0)
                        : cmode == ACC_PART ? CollideLDS::part_bytes(c->nv, hn[t], nsum, t == 0)
                                            : CollideLDS::bytes(c->nv, nsum, cmode, t == 0);
    // the attribute is per kernel, shared by every context: the largest
    // dynamic size the block size allows
    ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(kLdsBytes - collide_static_lds(cblock[t])));
    int per_cu = 0;
    if (ea == hipSuccess)
      ea = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, cblock[t], c->collide_lds[t]);
    if (ea == hipSuccess && per_cu < 1) ea = hipErrorInvalidConfiguration;
    c->collide_per_cu[t] = per_cu;
    int64_t cap = (int64_t)(per_cu < 1 ? 1 : per_cu) * (ncu < 1 ? 1 : ncu);
    if (hyb_rows) cap = std::min<int64_t>(cap, hyb_rows);
    c->collide_grid[t] = c->ncells < cap ? c->ncells : cap;
  }
  if (ea == hipSuccess && seq) {
    // the steps schedule where chains of dependent records are long against
    // the groups of 64 (few pairs per velocity node), else the groups; the
    // environment variable BOLTZ_SEQ_SCHEDULE=steps|groups overrides
    c->seq_sched = (double)p->n_pairs < 1.5 * (double)c->nv ? 1 : 0;
    if (const char* e = std::getenv("BOLTZ_SEQ_SCHEDULE")) {
      if (std::strcmp(e, "steps") == 0) c->seq_sched = 1;
      if (std::strcmp(e, "groups") == 0) c->seq_sched = 0;
    }
    const void* fn = c->seq_sched == 1 ? (const void*)seq_collide_kernel<1> : (const void*)seq_collide_kernel<0>;
    ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    int per_cu = 0;
    if (ea == hipSuccess)
      ea = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kSeqBlock, c->seq_lds);
    if (ea == hipSuccess && per_cu < 1) ea = hipErrorInvalidConfiguration;
    c->collide_per_cu[0] = c->collide_per_cu[1] = per_cu;
  }
  c->adj_supported = ea == hipSuccess && !seq && pick_adjoint(c->nv, nsum, c->adj_block, c->adj_fixed);
  for (int t = 0; t < 2 && ea == hipSuccess && c->adj_supported; ++t) {
    // the fixed-point layout when the runtime accepts its LDS size, else FP64 sums
    for (int attempt = 0; attempt < 2; ++attempt) {
      const void* fn = collide_adj_fn(c->adj_block, t == 1, c->adj_fixed[t]);
      c->adj_lds[t] = collide_adj_lds(c->nv, nsum, t == 0, c->adj_fixed[t]);
      ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->adj_lds[t]);
      int per_cu = 0;
      if (ea == hipSuccess)
        ea = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, c->adj_block, c->adj_lds[t]);
      if (ea == hipSuccess && per_cu < 1) ea = hipErrorInvalidConfiguration;
      if (ea == hipSuccess) {
        const int64_t cap = (int64_t)per_cu * (ncu < 1 ? 1 : ncu);
        c->adj_grid[t] = c->ncells < cap ? c->ncells : cap;
        break;
      }
      if (!c->adj_fixed[t]) break;
      (void)hipGetLastError();
      c->adj_fixed[t] = false;
    }
  }
  if (ea != hipSuccess) {
    boltz_destroy(c);
    return fail(nullptr, BOLTZ_EHIP, std::string("boltz_create: collide kernel set-up: ") + hipGetErrorString(ea));
  }
  *out = c;
  return BOLTZ_OK;
}

int boltz_query(const boltz_ctx* c, boltz_info* out) {
  if (!c || !out) return BOLTZ_EINVAL;
  out->ncells = c->ncells;
  out->nv = c->nv;
  out->dt = c->dt;
  out->K = c->K;
  out->W = c->W;
  out->qfac = c->qfac;
  out->device_bytes = (int64_t)c->dbytes;
  out->collide_layout = c->seq ? BOLTZ_LAYOUT_SEQUENTIAL : c->collide_mode;
  out->collide_block = c->seq ? 64 : c->collide_block[1];
  out->collide_lds_nodes = c->seq ? (int)c->nv
                           : (c->collide_mode == ACC_HYBRID || c->collide_mode == ACC_PART) ? c->hyb_n[1]
                           : (c->collide_mode == ACC_SPLIT ? (int)((c->nv + 1) / 2) : (int)c->nv);
  out->collide_per_cu = c->collide_per_cu[1];
  return BOLTZ_OK;
}

int boltz_axis_thresholds(const boltz_ctx* c, int axis, uint64_t* out) {
  if (!c || !out || axis < 0 || axis > 2) return BOLTZ_EINVAL;
  for (int i = 1; i < c->n[axis]; ++i) out[i - 1] = c->T[axis][i];
  return BOLTZ_OK;
}

// Rebuild the wall tables (Phi_w / Phi0 and the flux constants A, D) when the
// wall state differs from the one they were built for.
// The lid velocity and the side and top temperatures reach the kernel by
// value; the bottom faces' temperatures (a host array) are copied only when
// they change, and then only outside a stream capture (a captured copy would
// read host memory that no longer exists when the graph is replayed).
static int ensure_ratio(boltz_ctx* c, const WallArgs& W, const boltz_walls* walls, hipStream_t st) {
  std::vector<double> taub = bottom_taus(walls, c->p.nx);
  const bool same_b = c->ratio_valid && taub == c->ratio_taub;
  const bool same_w = c->ratio_valid && std::memcmp(&c->ratio_walls, &W, sizeof(WallArgs)) == 0;
  if (same_b && same_w) return BOLTZ_OK;
  int first = 0, count = 3 + c->p.nx;
  if (same_b) {
    // side walls (blocks 0, 1) and lid (block 2); the bottom tables stand
    const WallArgs& o = c->ratio_walls;
    const bool sides = o.tau[0] != W.tau[0] || o.tau[1] != W.tau[1];
    first = sides ? 0 : 2;
    count = sides ? 3 : 1;
  } else {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(c, BOLTZ_EINVAL,
                  "bottom-wall temperatures changed during a stream capture: make one call with the new walls "
                  "before capturing");
    // from pageable host memory: staged before the call returns
    hipError_t e = hipMemcpyAsync(const_cast<double*>(c->P.tau_b), taub.data(), taub.size() * sizeof(double),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "wall temperatures");
  }
  hipLaunchKernelGGL(wallconst_kernel, dim3(count), dim3(kWallConstBlock), 0, st, c->P, W, first);
  c->ratio_walls = W;
  c->ratio_taub = taub;
  c->ratio_valid = true;
  return BOLTZ_OK;
}

// Shared pair records that can be drawn in the last face launch: a table
// written directly by the sampler (no split-mode sort after it).
static bool samples_with_walls(const boltz_ctx* c) {
  return c->ngroups > 0 && c->p.n_pairs > 0 && c->collide_mode != ACC_SPLIT;
}

// The face densities; with sample_step >= 0 (and samples_with_walls) the
// records of that step are drawn in the last face launch.
static int launch_walls(boltz_ctx* c, const float* h, const WallArgs& W, const boltz_walls* walls,
                        hipStream_t st, int64_t sample_step = -1) {
  const int rc = ensure_ratio(c, W, walls, st);
  if (rc != BOLTZ_OK) return rc;
  auto launch = [&](auto kern, int nface) {
    const int per_xcd = (nface + 7) / 8;
    hipLaunchKernelGGL(kern, dim3(8 * per_xcd), dim3(kWallBlock), 0, st, c->P, h, nface, per_xcd);
  };
  // order 2: x faces first, then the y faces, which read the x-face
  // densities for their x-swept rows; the pair records go with the last
  // (and, for order 2, longer) launch
  const bool with_samples = sample_step >= 0 && samples_with_walls(c);
  auto launch_last = [&](auto kern, auto kern_s, int nface) {
    if (!with_samples) {
      launch(kern, nface);
      return;
    }
    const int per_xcd = (nface + 7) / 8;
    const int nb = (int)((c->p.n_pairs + kSampleBlock - 1) / kSampleBlock);
    const int nsum = c->n[0] + c->n[1] + c->n[2];
    hipLaunchKernelGGL(kern_s, dim3((unsigned)(8 * per_xcd + nb * c->ngroups)), dim3(kWallBlock),
                       TablesLDS::bytes(nsum, true), st, c->P, h, nface, per_xcd, nb, (uint32_t)sample_step,
                       c->tidx, c->tcoef, c->seq ? 0 : 1);
  };
  if (c->p.order == 2) {
    launch(wall_kernel<0>, 2 * c->p.ny);
    launch_last(wall_kernel<1>, wall_sample_kernel<1>, 2 * c->p.nx);
  } else {
    launch_last(wall_kernel<0>, wall_sample_kernel<0>, 2 * (c->p.nx + c->p.ny));
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "wall_kernel launch");
}

static int launch_stream(boltz_ctx* c, const float* hin, float* hout, hipStream_t st) {
  if (c->sstretched && c->n[2] % 4 != 0) {
    // stretched spatial cells (order 1): each cell's Courant numbers (the
    // vector kernel below takes them too)
    const int tiles_x = (c->p.nx + kTX - 1) / kTX, tiles_y = (c->p.ny + kTY - 1) / kTY;
    const int nchunks = (c->nv + kJ - 1) / kJ;
    const long long total = (long long)tiles_x * tiles_y * nchunks;
    const int per_xcd = (int)((total + 7) / 8);
    hipLaunchKernelGGL((stream_kernel<1, true>), dim3((unsigned)(8 * (long long)per_xcd)), dim3(kStreamBlock), 0, st,
                       c->P, hin, hout, tiles_x, tiles_y, nchunks, per_xcd);
  } else if (c->n[2] % 4 == 0) {
    // velocity groups of four share (jx, jy): vector kernel
    const int tiles_x = (c->p.nx + kTX4 - 1) / kTX4, tiles_y = (c->p.ny + kTY4 - 1) / kTY4;
    const long long total = stream4_units(c->p.nx, c->p.ny, c->nv);
    const int per_xcd = (int)((total + 7) / 8);
    const dim3 grid((unsigned)(8 * (long long)per_xcd));
    if (c->p.order == 2)
      hipLaunchKernelGGL(stream4_kernel<2>, grid, dim3(kStream4Block), 0, st, c->P, hin, hout, tiles_x, tiles_y,
                         (int)total, per_xcd);
    else
      hipLaunchKernelGGL(stream4_kernel<1>, grid, dim3(kStream4Block), 0, st, c->P, hin, hout, tiles_x, tiles_y,
                         (int)total, per_xcd);
  } else {
    const int tiles_x = (c->p.nx + kTX - 1) / kTX, tiles_y = (c->p.ny + kTY - 1) / kTY;
    const int nchunks = (c->nv + kJ - 1) / kJ;
    const long long total = (long long)tiles_x * tiles_y * nchunks;
    const int per_xcd = (int)((total + 7) / 8);
    const dim3 grid((unsigned)(8 * (long long)per_xcd));
    if (c->p.order == 2)
      hipLaunchKernelGGL(stream_kernel<2>, grid, dim3(kStreamBlock), 0, st, c->P, hin, hout, tiles_x, tiles_y,
                         nchunks, per_xcd);
    else
      hipLaunchKernelGGL(stream_kernel<1>, grid, dim3(kStreamBlock), 0, st, c->P, hin, hout, tiles_x, tiles_y,
                         nchunks, per_xcd);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "stream_kernel launch");
}

static RecordTables own_tables(const boltz_ctx* c) {
  const bool split = c->collide_mode == ACC_SPLIT;
  return RecordTables{c->tidx, c->tcoef, split ? c->sidx : c->tidx, split ? c->scoef : c->tcoef, c->sched};
}

extern "C++" template <int B, int M>
static void launch_collide_m(boltz_ctx* c, bool table, const float* hs, float* hout, uint32_t s32, uint32_t flags,
                             double* defect, hipStream_t st, const RecordTables& R) {
  const int t = table ? 1 : 0;
  const dim3 grid((unsigned)c->collide_grid[t]);
  const size_t lds = c->collide_lds[t];
  Params P = c->P;
  P.hyb_lo = c->hyb_lo[t];
  P.hyb_n = c->hyb_n[t];
  if (table)
    hipLaunchKernelGGL((collide_kernel<B, true, M>), grid, dim3(B), lds, st, P, hs, hout, s32, flags, defect,
                       R.tidx, R.tcoef);
  else if (P.continuous)
    hipLaunchKernelGGL((collide_kernel<B, false, M, 2>), grid, dim3(B), lds, st, P, hs, hout, s32, flags, defect,
                       R.tidx, R.tcoef);
  else
    hipLaunchKernelGGL((collide_kernel<B, false, M, 1>), grid, dim3(B), lds, st, P, hs, hout, s32, flags, defect,
                       R.tidx, R.tcoef);
}

extern "C++" template <int B>
static void launch_collide_b(boltz_ctx* c, bool table, const float* hs, float* hout, uint32_t s32, uint32_t flags,
                             double* defect, hipStream_t st, const RecordTables& R) {
  switch (c->collide_mode) {
    case ACC_HYBRID:
      if (B == 1024) launch_collide_m<1024, ACC_HYBRID>(c, table, hs, hout, s32, flags, defect, st, R);
      break;
    case ACC_PART:
      if (B == 1024) launch_collide_m<1024, ACC_PART>(c, table, hs, hout, s32, flags, defect, st, R);
      break;
    case ACC_FIXED: launch_collide_m<B, ACC_FIXED>(c, table, hs, hout, s32, flags, defect, st, R); break;
    case ACC_SPLIT: launch_collide_m<B, ACC_SPLIT>(c, table, hs, hout, s32, flags, defect, st, R); break;
    default: launch_collide_m<B, ACC_CAS>(c, table, hs, hout, s32, flags, defect, st, R); break;
  }
}

// Shared-sample mode: the pair records of every group for this step
// (ACC_SPLIT: then sorted by the velocity half of their targets).
static void launch_samples(boltz_ctx* c, uint32_t s32, hipStream_t st, const RecordTables& R) {
  if (c->ngroups > 0 && c->p.n_pairs > 0) {
    const int nsum = c->n[0] + c->n[1] + c->n[2];
    const dim3 grid((unsigned)((c->p.n_pairs + kSampleBlock - 1) / kSampleBlock), (unsigned)c->ngroups);
    // records in sample order for the sequential collision, else dealt to
    // lanes where no sort follows
    hipLaunchKernelGGL(sample_kernel, grid, dim3(kSampleBlock), TablesLDS::bytes(nsum, true), st, c->P, s32, R.sidx,
                       R.scoef, (R.sidx == R.tidx && !c->seq) ? 1 : 0);
    if (R.sidx != R.tidx)
      hipLaunchKernelGGL(split_sort_kernel, dim3((unsigned)c->ngroups), dim3(kSortBlock), 0, st, R.sidx, R.scoef,
                         R.tidx, R.tcoef, (int64_t)c->p.n_pairs, (unsigned)CollideLDS::half(c->nv));
  }
}

static void launch_samples(boltz_ctx* c, uint32_t s32, hipStream_t st) { launch_samples(c, s32, st, own_tables(c)); }

// The collision with the records in R (drawn: already written this step).
static int launch_collide_r(boltz_ctx* c, const float* hs, float* hout, int64_t step, uint32_t flags,
                            double* defect, hipStream_t st, bool drawn, const RecordTables& R) {
  const uint32_t s32 = (uint32_t)step;
  const bool table = c->ngroups > 0;
  if (!drawn) launch_samples(c, s32, st, R);
  if (c->seq) {
    // Alg. 3: the record levels of every sample group, then one wavefront
    // per cell
    const int64_t ngr = (c->p.n_pairs + kSeqGroup - 1) / kSeqGroup;
    const SeqSched S = SeqSched::carve(R.sched, ngr, c->ngroups);
    // the groups schedule keeps one level word per record at the start of
    // the same region
    uint16_t* lev = reinterpret_cast<uint16_t*>(R.sched);
    const dim3 grid((unsigned)c->ncells), block(kSeqBlock);
    if (c->seq_sched == 1) {
      if (ngr > 0) {
        hipLaunchKernelGGL(seq_level_kernel, dim3((unsigned)ngr, (unsigned)c->ngroups), dim3(kSeqGroup), 0, st,
                           R.tidx, R.tcoef, (int64_t)c->p.n_pairs, S);
        hipLaunchKernelGGL(seq_steps_kernel, dim3((unsigned)c->ngroups), dim3(kSeqGroup), 0, st,
                           (int64_t)c->p.n_pairs, S);
      }
      hipLaunchKernelGGL(seq_collide_kernel<1>, grid, block, c->seq_lds, st, c->P, c->vom, hs, hout, flags, defect,
                         R.tidx, R.tcoef, S, lev);
    } else {
      const int64_t ngr64 = (c->p.n_pairs + kSeqGroup64 - 1) / kSeqGroup64;
      if (ngr64 > 0)
        hipLaunchKernelGGL(seq_level64_kernel, dim3((unsigned)ngr64, (unsigned)c->ngroups), dim3(64), 0, st, R.tidx,
                           R.tcoef, (int64_t)c->p.n_pairs, lev);
      hipLaunchKernelGGL(seq_collide_kernel<0>, grid, block, c->seq_lds, st, c->P, c->vom, hs, hout, flags, defect,
                         R.tidx, R.tcoef, S, lev);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "seq_collide_kernel launch");
  }
  switch (c->collide_block[table ? 1 : 0]) {
    case 256: launch_collide_b<256>(c, table, hs, hout, s32, flags, defect, st, R); break;
    case 512: launch_collide_b<512>(c, table, hs, hout, s32, flags, defect, st, R); break;
    default: launch_collide_b<1024>(c, table, hs, hout, s32, flags, defect, st, R); break;
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "collide_kernel launch");
}

static int launch_collide(boltz_ctx* c, const float* hs, float* hout, int64_t step, uint32_t flags,
                          double* defect, hipStream_t st, bool drawn = false) {
  return launch_collide_r(c, hs, hout, step, flags, defect, st, drawn, own_tables(c));
}

static bool overlap(const void* a, const void* b, size_t n) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + n && y < x + n;
}

// boltz_stream; with sample_step >= 0 the shared records of that step are
// drawn with the face densities when possible (*drawn tells).
static int stream_step(boltz_ctx* c, const float* h_in, float* h_out, const boltz_walls* walls, hipStream_t st,
                       int64_t sample_step, bool* drawn) {
  if (!c) return BOLTZ_EINVAL;
  if (!h_in || !h_out) return fail(c, BOLTZ_EINVAL, "boltz_stream: null buffer");
  const size_t bytes = (size_t)c->ncells * c->nv * sizeof(float);
  if (overlap(h_in, h_out, bytes)) return fail(c, BOLTZ_EINVAL, "boltz_stream: h_in and h_out overlap");
  const bool cavity = c->p.bc == BOLTZ_BC_CAVITY;
  if (cavity && !walls_ok(walls, c->p.nx)) return fail(c, BOLTZ_EINVAL, "boltz_stream: cavity needs valid walls");
  int rc = BOLTZ_OK;
  if (cavity) rc = launch_walls(c, h_in, make_walls(walls), walls, st, sample_step);
  if (drawn) *drawn = cavity && sample_step >= 0 && samples_with_walls(c);
  if (rc == BOLTZ_OK) rc = launch_stream(c, h_in, h_out, st);
  return rc;
}

int boltz_stream(boltz_ctx* c, const float* h_in, float* h_out, const boltz_walls* walls, void* stream) {
  return stream_step(c, h_in, h_out, walls, static_cast<hipStream_t>(stream), -1, nullptr);
}

int boltz_collide(boltz_ctx* c, const float* h_s, float* h_out, int64_t step, uint32_t flags, double* defect,
                  void* stream) {
  if (!c) return BOLTZ_EINVAL;
  if (!h_s || !h_out) return fail(c, BOLTZ_EINVAL, "boltz_collide: null buffer");
  const size_t bytes = (size_t)c->ncells * c->nv * sizeof(float);
  if (h_s != h_out && overlap(h_s, h_out, bytes))
    return fail(c, BOLTZ_EINVAL, "boltz_collide: h_s and h_out partially overlap");
  if (flags & ~(uint32_t)BOLTZ_NO_CORRECTION) return fail(c, BOLTZ_EINVAL, "boltz_collide: unknown flag");
  return launch_collide(c, h_s, h_out, step, flags, defect, static_cast<hipStream_t>(stream));
}

int boltz_collide_noalloc(boltz_ctx* c, const float* h_s, float* h_out, int64_t step, uint32_t flags,
                          double* defect, void* stream) {
  if (!c) return BOLTZ_EINVAL;
  if (!h_s || !h_out) return fail(c, BOLTZ_EINVAL, "boltz_collide_noalloc: null buffer");
  const size_t bytes = (size_t)c->ncells * c->nv * sizeof(float);
  if (h_s != h_out && overlap(h_s, h_out, bytes))
    return fail(c, BOLTZ_EINVAL, "boltz_collide_noalloc: h_s and h_out partially overlap");
  if (flags & ~(uint32_t)BOLTZ_NO_CORRECTION) return fail(c, BOLTZ_EINVAL, "boltz_collide_noalloc: unknown flag");
  RecordTables R{nullptr, nullptr, nullptr, nullptr};
  if (c->ngroups > 0 && c->p.n_pairs > 0) {
    if (!c->scratch) return fail(c, BOLTZ_EHIP, "boltz_collide_noalloc: no device address of the record scratch");
    // one table: n index pairs (256-byte aligned), then n coefficient sets;
    // the split layout needs a second one for the sampler's unsorted output
    const size_t n = (size_t)c->ngroups * (size_t)c->p.n_pairs;
    const bool split = c->collide_mode == ACC_SPLIT;
    const size_t one = align256(n * sizeof(uint2)) + n * sizeof(float4);
    // the sequential collision also keeps its step schedule
    const size_t nsch = c->seq ? SeqSched::bytes((c->p.n_pairs + kSeqGroup - 1) / kSeqGroup, c->ngroups) : 0;
    const size_t need = split ? align256(one) + one : (c->seq ? align256(one) + nsch : one);
    if (need > kScratchBytes)
      return fail(c, BOLTZ_EINVAL,
                  "boltz_collide_noalloc: " + std::to_string(need) + " bytes of shared-sample records exceed the " +
                      std::to_string(kScratchBytes) + "-byte scratch (about " +
                      std::to_string(kScratchBytes / ((split ? 2 : 1) * 24)) + " records per step at most)");
    unsigned char* p = c->scratch;
    R.tidx = reinterpret_cast<uint2*>(p);
    R.tcoef = reinterpret_cast<float4*>(p + align256(n * sizeof(uint2)));
    R.sidx = R.tidx;
    R.scoef = R.tcoef;
    if (split) {
      unsigned char* q = p + align256(one);
      R.sidx = reinterpret_cast<uint2*>(q);
      R.scoef = reinterpret_cast<float4*>(q + align256(n * sizeof(uint2)));
    }
    if (c->seq) R.sched = p + align256(one);
  }
  return launch_collide_r(c, h_s, h_out, step, flags, defect, static_cast<hipStream_t>(stream), false, R);
}

int boltz_step(boltz_ctx* c, const float* h_in, float* h_out, const boltz_walls* walls, int64_t step,
               void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  bool drawn = false;
  const int rc = stream_step(c, h_in, h_out, walls, st, step, &drawn);
  if (rc != BOLTZ_OK) return rc;
  return launch_collide(c, h_out, h_out, step, 0u, nullptr, st, drawn);
}

int boltz_moments(boltz_ctx* c, const float* h, const boltz_walls* walls, double* mom, double* lid_shear,
                  void* stream) {
  if (!c) return BOLTZ_EINVAL;
  if (!h || !mom) return fail(c, BOLTZ_EINVAL, "boltz_moments: null buffer");
  if (lid_shear && (c->p.bc != BOLTZ_BC_CAVITY || !walls_ok(walls, c->p.nx)))
    return fail(c, BOLTZ_EINVAL, "boltz_moments: lid shear needs a cavity and valid walls");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const WallArgs W = make_walls(walls);
  if (lid_shear) {
    const int rc = ensure_ratio(c, W, walls, st);
    if (rc != BOLTZ_OK) return rc;
  }
  hipLaunchKernelGGL(moments_kernel, dim3((unsigned)c->ncells), dim3(kMomentsBlock), 0, st, c->P, W, h, mom,
                     lid_shear ? 1 : 0);
  if (lid_shear) hipLaunchKernelGGL(lid_reduce_kernel, dim3(1), dim3(64), 0, st, c->P, lid_shear);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "moments_kernel launch");
}

}  // extern "C"

// ------------------------------------------------------------- adjoint --
// Reverse mode of the streaming step whose face densities P.nw are current:
// lo (adjoint of the streamed state) -> li.  Order 2: y sweep transposed
// into tmp, then x sweep into li (li may equal lo); order 1: li != lo.
// Wall-parameter partials go to grad (when not NULL).
static int launch_stream_adj(boltz_ctx* c, const WallArgs& W, const double* lo, double* li, double* tmp,
                             double* grad, hipStream_t st) {
  const bool cavity = c->p.bc == BOLTZ_BC_CAVITY;
  const int nx = c->p.nx, ny = c->p.ny;
  const int nchunks = (c->nv + kSweepAdjBlock - 1) / kSweepAdjBlock;
  auto walls_adj = [&](const double* lam, int f0, int nface) {
    const int per_xcd = (nface + 7) / 8;
    hipLaunchKernelGGL(wall_adj_kernel, dim3(8 * per_xcd), dim3(kWallAdjBlock), 0, st, c->P, W, lam, c->lnw,
                       c->gpart, f0, nface, per_xcd);
  };
  auto sweep = [&](auto kern, const double* in, double* out, int nlines) {
    const long long units = (long long)nlines * nchunks;
    const int per_xcd = (int)((units + 7) / 8);
    hipLaunchKernelGGL(kern, dim3((unsigned)(8 * (long long)per_xcd)), dim3(kSweepAdjBlock), 0, st, c->P, in, out,
                       c->lnw, nchunks, per_xcd);
  };
  if (c->p.order == 2) {
    // y faces and the y sweep read the adjoint of the y-sweep output; the x
    // faces and the x sweep that of the x-swept state
    if (cavity) walls_adj(lo, 2 * ny, 2 * nx);
    sweep(sweep_adj_kernel<1>, lo, tmp, nx);
    if (cavity) walls_adj(tmp, 0, 2 * ny);
    sweep(sweep_adj_kernel<0>, tmp, li, ny);
  } else {
    if (cavity) walls_adj(lo, 0, 2 * (nx + ny));
    const int nc = (c->nv + kOrder1AdjBlock - 1) / kOrder1AdjBlock;
    hipLaunchKernelGGL(order1_adj_kernel, dim3((unsigned)(c->ncells * nc)), dim3(kOrder1AdjBlock), 0, st, c->P, lo,
                       li, c->lnw, nc);
  }
  if (cavity && grad) hipLaunchKernelGGL(grad_reduce_kernel, dim3(1), dim3(256), 0, st, c->P, c->gpart, grad, 3);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "stream adjoint launch");
}

extern "C++" template <int B, bool TABLE, bool FIXED>
static void launch_collide_adj_v(boltz_ctx* c, const float* hs, const double* lo, double* ls, uint32_t s32,
                                 uint32_t flags, hipStream_t st) {
  const int t = TABLE ? 1 : 0;
  hipLaunchKernelGGL((collide_adj_kernel<B, TABLE, FIXED>), dim3((unsigned)c->adj_grid[t]), dim3(B), c->adj_lds[t],
                     st, c->P, hs, lo, ls, s32, flags, c->tidx, c->tcoef);
}

extern "C++" template <int B>
static void launch_collide_adj_b(boltz_ctx* c, bool table, const float* hs, const double* lo, double* ls,
                                 uint32_t s32, uint32_t flags, hipStream_t st) {
  const bool fixed = c->adj_fixed[table ? 1 : 0];
  if (table) {
    if (fixed) launch_collide_adj_v<B, true, true>(c, hs, lo, ls, s32, flags, st);
    else launch_collide_adj_v<B, true, false>(c, hs, lo, ls, s32, flags, st);
  } else {
    if (fixed) launch_collide_adj_v<B, false, true>(c, hs, lo, ls, s32, flags, st);
    else launch_collide_adj_v<B, false, false>(c, hs, lo, ls, s32, flags, st);
  }
}

static int launch_collide_adj(boltz_ctx* c, const float* hs, const double* lo, double* ls, int64_t step,
                              uint32_t flags, hipStream_t st) {
  const uint32_t s32 = (uint32_t)step;
  const bool table = c->ngroups > 0;
  launch_samples(c, s32, st);
  if (c->adj_block == 256) launch_collide_adj_b<256>(c, table, hs, lo, ls, s32, flags, st);
  else launch_collide_adj_b<512>(c, table, hs, lo, ls, s32, flags, st);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "collide adjoint launch");
}

extern "C" {

int boltz_stream_adjoint(boltz_ctx* c, const float* h_in, const double* lam_out, double* lam_in, double* grad_walls,
                         const boltz_walls* walls, void* stream) {
  if (!c) return BOLTZ_EINVAL;
  if (!h_in || !lam_out || !lam_in) return fail(c, BOLTZ_EINVAL, "boltz_stream_adjoint: null buffer");
  const size_t bytes = (size_t)c->ncells * c->nv * sizeof(double);
  if (overlap(lam_out, lam_in, bytes)) return fail(c, BOLTZ_EINVAL, "boltz_stream_adjoint: lam_out and lam_in overlap");
  const bool cavity = c->p.bc == BOLTZ_BC_CAVITY;
  if (cavity && !walls_ok(walls, c->p.nx))
    return fail(c, BOLTZ_EINVAL, "boltz_stream_adjoint: cavity needs valid walls");
  if (c->p.order == 2 && !c->adj_lam)
    return fail(c, BOLTZ_EINVAL, "boltz_stream_adjoint: order 2 needs a context created with BOLTZ_WITH_ADJOINT");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const WallArgs W = make_walls(walls);
  int rc = BOLTZ_OK;
  if (cavity) rc = launch_walls(c, h_in, W, walls, st);
  if (rc == BOLTZ_OK) rc = launch_stream_adj(c, W, lam_out, lam_in, c->adj_lam, grad_walls, st);
  return rc;
}

int boltz_collide_adjoint(boltz_ctx* c, const float* h_s, const double* lam_out, double* lam_s, int64_t step,
                          uint32_t flags, void* stream) {
  if (!c) return BOLTZ_EINVAL;
  if (!h_s || !lam_out || !lam_s) return fail(c, BOLTZ_EINVAL, "boltz_collide_adjoint: null buffer");
  const size_t bytes = (size_t)c->ncells * c->nv * sizeof(double);
  if (lam_out != lam_s && overlap(lam_out, lam_s, bytes))
    return fail(c, BOLTZ_EINVAL, "boltz_collide_adjoint: lam_out and lam_s partially overlap");
  if (flags & ~(uint32_t)BOLTZ_NO_CORRECTION) return fail(c, BOLTZ_EINVAL, "boltz_collide_adjoint: unknown flag");
  if (!c->adj_supported)
    return fail(c, BOLTZ_EUNSUPPORTED, "boltz_collide_adjoint: velocity grid too large for the adjoint's LDS layout");
  return launch_collide_adj(c, h_s, lam_out, lam_s, step, flags, static_cast<hipStream_t>(stream));
}

int boltz_step_adjoint(boltz_ctx* c, const float* h_in, const double* lam_out, double* lam_in, double* grad_walls,
                       const boltz_walls* walls, int64_t step, void* stream) {
  if (!c) return BOLTZ_EINVAL;
  if (!h_in || !lam_out || !lam_in) return fail(c, BOLTZ_EINVAL, "boltz_step_adjoint: null buffer");
  const size_t bytes = (size_t)c->ncells * c->nv * sizeof(double);
  if (lam_out != lam_in && overlap(lam_out, lam_in, bytes))
    return fail(c, BOLTZ_EINVAL, "boltz_step_adjoint: lam_out and lam_in partially overlap");
  if (!c->adj_hs || !c->adj_lam)
    return fail(c, BOLTZ_EINVAL, "boltz_step_adjoint: context not created with BOLTZ_WITH_ADJOINT");
  if (!c->adj_supported)
    return fail(c, BOLTZ_EUNSUPPORTED, "boltz_step_adjoint: velocity grid too large for the adjoint's LDS layout");
  const bool cavity = c->p.bc == BOLTZ_BC_CAVITY;
  if (cavity && !walls_ok(walls, c->p.nx))
    return fail(c, BOLTZ_EINVAL, "boltz_step_adjoint: cavity needs valid walls");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const WallArgs W = make_walls(walls);
  // forward streaming again (also leaves the face densities of h_in in P.nw)
  int rc = BOLTZ_OK;
  if (cavity) rc = launch_walls(c, h_in, W, walls, st);
  if (rc == BOLTZ_OK) rc = launch_stream(c, h_in, c->adj_hs, st);
  if (rc != BOLTZ_OK) return rc;
  if (c->p.order == 2) {
    // collision adjoint into lam_in (in place when it is lam_out), then the
    // sweeps through the scratch back into lam_in
    rc = launch_collide_adj(c, c->adj_hs, lam_out, lam_in, step, 0u, st);
    if (rc == BOLTZ_OK) rc = launch_stream_adj(c, W, lam_in, lam_in, c->adj_lam, grad_walls, st);
  } else {
    rc = launch_collide_adj(c, c->adj_hs, lam_out, c->adj_lam, step, 0u, st);
    if (rc == BOLTZ_OK) rc = launch_stream_adj(c, W, c->adj_lam, lam_in, nullptr, grad_walls, st);
  }
  return rc;
}

int boltz_lid_shear_adjoint(boltz_ctx* c, const float* h, const boltz_walls* walls, double weight, double* lam,
                            double* grad_walls, void* stream) {
  if (!c) return BOLTZ_EINVAL;
  if (!h || !lam) return fail(c, BOLTZ_EINVAL, "boltz_lid_shear_adjoint: null buffer");
  if (c->p.bc != BOLTZ_BC_CAVITY || !walls_ok(walls, c->p.nx) || !std::isfinite(weight))
    return fail(c, BOLTZ_EINVAL, "boltz_lid_shear_adjoint: needs a cavity, valid walls and a finite weight");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const WallArgs W = make_walls(walls);
  const int rc = ensure_ratio(c, W, walls, st);
  if (rc != BOLTZ_OK) return rc;
  hipLaunchKernelGGL(lid_adj_kernel, dim3((unsigned)c->p.nx), dim3(kLidAdjBlock), 0, st, c->P, W, h, weight, lam,
                     c->gpart);
  if (grad_walls) hipLaunchKernelGGL(lid_grad_kernel, dim3(1), dim3(64), 0, st, c->P, c->gpart, grad_walls);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "lid shear adjoint launch");
}

int boltz_debug_pairs(boltz_ctx* c, int64_t cell, int64_t step, int64_t m0, int64_t count, int32_t* idx4,
                      double* q, uint32_t* words) {
  if (!c) return BOLTZ_EINVAL;
  if (cell < 0 || cell >= c->ncells || m0 < 0 || count < 0 || m0 + count > ((int64_t)1 << 31) || !idx4 || !q)
    return fail(c, BOLTZ_EINVAL, "boltz_debug_pairs: invalid argument");
  if (count == 0) return BOLTZ_OK;
  const size_t bi = (size_t)count * 4 * sizeof(int32_t), bq = (size_t)count * sizeof(double),
               bw = words ? (size_t)count * 4 * sizeof(uint32_t) : 0;
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bi + bq + bw + 64);
  if (e != hipSuccess) return hip_fail(c, e, "boltz_debug_pairs: hipMalloc");
  unsigned char* b = static_cast<unsigned char*>(d);
  int32_t* d_idx = reinterpret_cast<int32_t*>(b);
  double* d_q = reinterpret_cast<double*>(b + ((bi + 7) & ~(size_t)7));
  uint32_t* d_w = words ? reinterpret_cast<uint32_t*>(b + ((bi + 7) & ~(size_t)7) + bq) : nullptr;
  const int nsum = c->n[0] + c->n[1] + c->n[2];
  const size_t lds = TablesLDS::bytes(nsum, true);
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(debug_pairs_kernel, dim3(blocks), dim3(256), lds, 0, c->P, cell, (uint32_t)step, m0, count,
                     d_idx, d_q, d_w);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(idx4, d_idx, bi, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(q, d_q, bq, hipMemcpyDeviceToHost);
  if (e == hipSuccess && words) e = hipMemcpy(words, d_w, bw, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "boltz_debug_pairs");
}

int boltz_read_status(boltz_ctx* c, uint32_t* out, int clear, void* stream) {
  if (!c || !out) return BOLTZ_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(out, c->P.status, 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && clear) e = hipMemset(c->P.status, 0, 4);
  return e == hipSuccess ? BOLTZ_OK : hip_fail(c, e, "boltz_read_status");
}

}  // extern "C"

// --------------------------------------------------------------- batches --
namespace {

__global__ void set_step_kernel(uint32_t* step, uint32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step = v;
}

__global__ void advance_step_kernel(uint32_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1u;
}

const void* collide_batch_fn(int block, int pu) {
  if (block == 256) return pu == 2 ? (const void*)collide_batch_kernel<256, 2> : (const void*)collide_batch_kernel<256, 4>;
  if (block == 512) return pu == 2 ? (const void*)collide_batch_kernel<512, 2> : (const void*)collide_batch_kernel<512, 4>;
  return pu == 2 ? (const void*)collide_batch_kernel<1024, 2> : (const void*)collide_batch_kernel<1024, 4>;
}

// A class of a batch: its problems with one velocity grid.  The class's
// cells (items item0 .. item0 + nitems - 1, by decreasing cost) are one
// collide launch with settings of its own: block size, shared records per
// thread in flight (pu) and workgroups (spread 0: one per resident slot,
// 1: two per slot, 2: one per cell).
struct BatchClass {
  int nv3[3] = {0, 0, 0};
  int problems = 0;
  int64_t cells = 0, pair_cells = 0;
  int item0 = 0, nitems = 0;
  size_t lds = 0;
  bool ok[3] = {false, false, false};  // 256, 512, 1024 threads fit
  int64_t cap[3] = {0, 0, 0};          // resident workgroups (all CUs)
  int block = 512, pu = 4, spread = 0;
  bool part = false;                   // ACC_PART: 1024 threads, spread 0 or 1 (the global rows)
  double ms = 0.0;                     // ms per launch measured by the tuner
};

int block_index(int block) { return block == 256 ? 0 : (block == 512 ? 1 : 2); }

int64_t class_grid(const BatchClass& k) {
  const int64_t cap = k.cap[block_index(k.block)];
  const int64_t g = k.spread == 0 ? cap : (k.spread == 1 ? 2 * cap : (int64_t)k.nitems);
  return std::max<int64_t>(1, std::min<int64_t>(g, k.nitems));
}

}  // namespace

struct boltz_batch {
  std::vector<boltz_ctx*> ctx;
  std::vector<int64_t> hoff;
  int count = 0;
  int order = 2;
  bool any_cavity = false;
  int device = 0;
  void* dmem = nullptr;
  size_t dbytes = 0;
  BatchCav* cavs = nullptr;
  // first unit of each problem in the batched launches: x faces (all faces
  // for order 1), y faces, stream units, sample blocks, sort workgroups
  int* start[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int total[5] = {0, 0, 0, 0, 0};
  int2* items = nullptr;
  int nitems = 0;
  std::vector<BatchClass> cls;
  // stream work units per problem for the 32 x 4 tile shape (start[2], total[2]: 16 x 8)
  int* start_b = nullptr;
  int total_b = 0;
  int stile = 0;  // stream tile shape in use: 0 = 16 x 8, 1 = 32 x 4
  uint32_t* step_dev = nullptr;
  int64_t nodes = 0;
  int64_t pair_cells = 0;
  size_t sample_lds = 0;
  std::string err;
};

namespace {

thread_local std::string g_batch_error;

int bfail(boltz_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg; else g_batch_error = msg;
  return code;
}

// Launch one class's collision, hin -> hout (the batched step: in place).
void launch_class(const boltz_batch* b, const BatchClass& k, const float* hin, float* hout, hipStream_t st) {
  const dim3 grid((unsigned)class_grid(k));
  const int2* it = b->items + k.item0;
#define BOLTZ_CLASS_LAUNCH(B, U)                                                                              \
  hipLaunchKernelGGL((collide_batch_kernel<B, U>), grid, dim3(B), k.lds, st, b->cavs, it, k.nitems, hin, hout,   \
                     b->step_dev)
  if (k.block == 256) {
    if (k.pu == 2) BOLTZ_CLASS_LAUNCH(256, 2); else BOLTZ_CLASS_LAUNCH(256, 4);
  } else if (k.block == 512) {
    if (k.pu == 2) BOLTZ_CLASS_LAUNCH(512, 2); else BOLTZ_CLASS_LAUNCH(512, 4);
  } else {
    if (k.pu == 2) BOLTZ_CLASS_LAUNCH(1024, 2); else BOLTZ_CLASS_LAUNCH(1024, 4);
  }
#undef BOLTZ_CLASS_LAUNCH
}

}  // namespace

extern "C" {

const char* boltz_batch_last_error(const boltz_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

void boltz_batch_destroy(boltz_batch* b) {
  if (!b) return;
  for (boltz_ctx* c : b->ctx) boltz_destroy(c);
  if (b->dmem) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(b->device);
    (void)hipFree(b->dmem);
    (void)hipSetDevice(cur);
  }
  delete b;
}

int boltz_batch_create(const boltz_problem* problems, int count, boltz_batch** out) {
  if (!problems || !out || count < 1 || count > 4096)
    return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: need 1..4096 problems and an output pointer");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (problems[i].order != problems[0].order)
      return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: all problems need the same streaming order");
    if (problems[i].nv[2] % 4 != 0)
      return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: batched streaming needs nv[2] % 4 == 0");
    if ((int64_t)problems[i].nx * problems[i].ny >= ((int64_t)1 << 31))
      return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: too many cells in one problem");
    if (problems[i].flags & BOLTZ_SEQUENTIAL_UPDATE)
      return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: batches take the Jacobi collision only");
    if ((problems[i].rx != 0.0 && problems[i].rx != 1.0) || (problems[i].ry != 0.0 && problems[i].ry != 1.0))
      return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: batches take uniform spatial cells only");
  }
  boltz_batch* b = new (std::nothrow) boltz_batch;
  if (!b) return bfail(nullptr, BOLTZ_ENOMEM, "boltz_batch_create: out of host memory");
  b->count = count;
  b->order = problems[0].order;
  (void)hipGetDevice(&b->device);
  for (int i = 0; i < count; ++i) {
    boltz_ctx* c = nullptr;
    const int rc = boltz_create(&problems[i], &c);
    if (rc != BOLTZ_OK) {
      const std::string msg = "boltz_batch_create: problem " + std::to_string(i) + ": " + g_create_error;
      boltz_batch_destroy(b);
      return bfail(nullptr, rc, msg);
    }
    b->ctx.push_back(c);
  }
  // ---- descriptors, launch ranges, work items
  std::vector<BatchCav> cavs(count);
  std::vector<int> st[5], stb(count + 1, 0);
  for (int k = 0; k < 5; ++k) st[k].assign(count + 1, 0);
  std::vector<double> cost(count);
  std::vector<int> cls_of(count);
  int64_t off = 0;
  size_t slds_max = 0;
  for (int i = 0; i < count; ++i) {
    const boltz_ctx* c = b->ctx[i];
    BatchCav& C = cavs[i];
    std::memset(&C, 0, sizeof(C));
    C.P = c->P;
    C.hoff = off;
    C.tidx = c->tidx;
    C.tcoef = c->tcoef;
    // a problem whose single-problem collision uses the partial-tile layout
    // keeps it (its records unsorted); the others take the batch layouts
    const bool part = c->collide_mode == ACC_PART;
    const int tv = c->ngroups > 0 ? 1 : 0;
    C.P.hyb_lo = c->hyb_lo[tv];
    C.P.hyb_n = c->hyb_n[tv];
    C.sidx = part ? c->tidx : c->sidx;
    C.scoef = part ? c->tcoef : c->scoef;
    C.mode = part ? ACC_PART : c->batch_mode;
    b->hoff.push_back(off);
    off += c->ncells * (int64_t)c->nv;
    const bool cavity = c->p.bc == BOLTZ_BC_CAVITY;
    b->any_cavity = b->any_cavity || cavity;
    const int nx = c->p.nx, ny = c->p.ny;
    const int nf0 = !cavity ? 0 : (b->order == 2 ? 2 * ny : 2 * (nx + ny));
    const int nf1 = (cavity && b->order == 2) ? 2 * nx : 0;
    const int64_t units = stream4_units(nx, ny, c->nv);
    const int64_t units_b = stream4_units(nx, ny, c->nv, kTX4b, kTY4b);
    if ((int64_t)stb[i] + units_b >= ((int64_t)1 << 31) / 8) {
      boltz_batch_destroy(b);
      return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: batch too large for one launch per phase");
    }
    stb[i + 1] = stb[i] + (int)units_b;
    const int64_t sblocks =
        (c->ngroups > 0 && c->p.n_pairs > 0) ? c->ngroups * ((c->p.n_pairs + kSampleBlock - 1) / kSampleBlock) : 0;
    const int64_t sorts = (!part && c->sidx != c->tidx) ? c->ngroups : 0;
    const int64_t nxt[5] = {(int64_t)st[0][i] + nf0, (int64_t)st[1][i] + nf1, (int64_t)st[2][i] + units,
                            (int64_t)st[3][i] + sblocks, (int64_t)st[4][i] + sorts};
    for (int k = 0; k < 5; ++k) {
      if (nxt[k] >= ((int64_t)1 << 31) / 8) {
        boltz_batch_destroy(b);
        return bfail(nullptr, BOLTZ_EINVAL, "boltz_batch_create: batch too large for one launch per phase");
      }
      st[k][i + 1] = (int)nxt[k];
    }
    const int nsum = c->n[0] + c->n[1] + c->n[2];
    const bool table = c->ngroups > 0;
    // class: the problems with this velocity grid
    int k = 0;
    while (k < (int)b->cls.size() && !(b->cls[k].nv3[0] == c->n[0] && b->cls[k].nv3[1] == c->n[1] &&
                                       b->cls[k].nv3[2] == c->n[2]))
      ++k;
    if (k == (int)b->cls.size()) {
      b->cls.emplace_back();
      for (int a = 0; a < 3; ++a) b->cls[k].nv3[a] = c->n[a];
    }
    BatchClass& K = b->cls[k];
    cls_of[i] = k;
    K.problems += 1;
    K.cells += c->ncells;
    K.pair_cells += c->ncells * c->p.n_pairs;
    K.part = part;
    K.lds = std::max(K.lds, part ? CollideLDS::part_bytes(c->nv, c->hyb_n[tv], nsum, !table)
                                 : CollideLDS::bytes(c->nv, nsum, c->batch_mode, !table));
    if (table) slds_max = std::max(slds_max, TablesLDS::bytes(nsum, true));
    // relative cost of one cell: pair loop (drawn pairs cost more) plus the node phases
    cost[i] = (double)c->p.n_pairs * (table ? 1.0 : 3.0) *
                  ((part || c->batch_mode == ACC_FIXED) ? 1.0 : (c->batch_mode == ACC_SPLIT ? 1.3 : 4.0)) +
              40.0 * c->nv;
    b->pair_cells += c->ncells * c->p.n_pairs;
  }
  b->nodes = off;
  for (int k = 0; k < 5; ++k) b->total[k] = st[k][count];
  b->total_b = stb[count];
  // work items grouped by class, by decreasing cost within a class
  std::vector<int2> items;
  for (int i = 0; i < count; ++i)
    for (int64_t cell = 0; cell < b->ctx[i]->ncells; ++cell) items.push_back(make_int2(i, (int)cell));
  std::stable_sort(items.begin(), items.end(), [&](const int2& x, const int2& y) {
    return cls_of[x.x] != cls_of[y.x] ? cls_of[x.x] < cls_of[y.x] : cost[x.x] > cost[y.x];
  });
  b->nitems = (int)items.size();
  for (size_t m = 0; m < items.size(); ++m) {
    BatchClass& K = b->cls[cls_of[items[m].x]];
    if (K.nitems++ == 0) K.item0 = (int)m;
  }
  b->sample_lds = slds_max;
  // ---- one device allocation
  size_t o = 0;
  const size_t o_cavs = o; o = align256(o + sizeof(BatchCav) * count);
  size_t o_st[5];
  for (int k = 0; k < 5; ++k) { o_st[k] = o; o = align256(o + sizeof(int) * (count + 1)); }
  const size_t o_stb = o; o = align256(o + sizeof(int) * (count + 1));
  const size_t o_items = o; o = align256(o + sizeof(int2) * items.size());
  const size_t o_step = o; o = align256(o + 4);
  hipError_t e = hipMalloc(&b->dmem, o);
  if (e != hipSuccess) {
    boltz_batch_destroy(b);
    return bfail(nullptr, BOLTZ_ENOMEM, std::string("boltz_batch_create: hipMalloc: ") + hipGetErrorString(e));
  }
  b->dbytes = o;
  unsigned char* base = static_cast<unsigned char*>(b->dmem);
  b->cavs = reinterpret_cast<BatchCav*>(base + o_cavs);
  for (int k = 0; k < 5; ++k) b->start[k] = reinterpret_cast<int*>(base + o_st[k]);
  b->start_b = reinterpret_cast<int*>(base + o_stb);
  b->items = reinterpret_cast<int2*>(base + o_items);
  b->step_dev = reinterpret_cast<uint32_t*>(base + o_step);
  e = hipMemcpy(b->cavs, cavs.data(), sizeof(BatchCav) * count, hipMemcpyHostToDevice);
  for (int k = 0; k < 5 && e == hipSuccess; ++k)
    e = hipMemcpy(b->start[k], st[k].data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->start_b, stb.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->step_dev, 0, 4);
  // ---- collide launch set-up for each block size whose LDS fits
  int ncu = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e == hipSuccess && slds_max > 0)
    e = hipFuncSetAttribute((const void*)sample_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)slds_max);
  const int blocks[3] = {256, 512, 1024};
  for (int t = 0; t < 3 && e == hipSuccess; ++t)
    for (int pu = 2; pu <= 4 && e == hipSuccess; pu += 2)
      e = hipFuncSetAttribute(collide_batch_fn(blocks[t], pu), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(kLdsBytes - collide_static_lds(blocks[t])));
  for (BatchClass& K : b->cls) {
    for (int t = 0; t < 3 && e == hipSuccess; ++t) {
      if (K.lds + collide_static_lds(blocks[t]) > kLdsBytes || (K.part && blocks[t] != 1024)) continue;
      int per_cu = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, collide_batch_fn(blocks[t], 4), blocks[t], K.lds);
      if (e != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        e = hipSuccess;
        continue;
      }
      K.ok[t] = true;
      K.cap[t] = (int64_t)per_cu * (ncu < 1 ? 1 : ncu);
      // the partial-tile layout's global rows: two per CU, one per workgroup
      if (K.part) K.cap[t] = std::min<int64_t>(K.cap[t], ncu < 1 ? 1 : ncu);
    }
    K.block = K.ok[1] ? 512 : (K.ok[0] ? 256 : 1024);
    if (e == hipSuccess && !K.ok[block_index(K.block)]) {
      boltz_batch_destroy(b);
      return bfail(nullptr, BOLTZ_EUNSUPPORTED, "boltz_batch_create: no collide block size fits a class's LDS");
    }
  }
  if (e != hipSuccess) {
    boltz_batch_destroy(b);
    return bfail(nullptr, BOLTZ_EHIP, std::string("boltz_batch_create: ") + hipGetErrorString(e));
  }
  *out = b;
  return BOLTZ_OK;
}

int boltz_batch_query(const boltz_batch* b, boltz_batch_info* out) {
  if (!b || !out) return BOLTZ_EINVAL;
  out->count = b->count;
  out->nodes = b->nodes;
  out->pair_cells = b->pair_cells;
  // the block size of the class with the most pair-cells
  const BatchClass* big = nullptr;
  for (const BatchClass& K : b->cls)
    if (!big || K.pair_cells > big->pair_cells) big = &K;
  out->collide_block = big ? big->block : 0;
  out->classes = (int32_t)b->cls.size();
  out->stream_tile[0] = b->stile == 0 ? kTX4 : kTX4b;
  out->stream_tile[1] = b->stile == 0 ? kTY4 : kTY4b;
  out->reserved = 0;
  int64_t bytes = (int64_t)b->dbytes;
  for (const boltz_ctx* c : b->ctx) bytes += (int64_t)c->dbytes;
  out->device_bytes = bytes;
  return BOLTZ_OK;
}

int boltz_batch_offsets(const boltz_batch* b, int64_t* offsets) {
  if (!b || !offsets) return BOLTZ_EINVAL;
  for (int i = 0; i < b->count; ++i) offsets[i] = b->hoff[i];
  return BOLTZ_OK;
}

boltz_ctx* boltz_batch_problem(boltz_batch* b, int index) {
  if (!b || index < 0 || index >= b->count) return nullptr;
  return b->ctx[index];
}

int boltz_batch_set_step(boltz_batch* b, int64_t step, void* stream) {
  if (!b) return BOLTZ_EINVAL;
  hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), b->step_dev,
                     (uint32_t)step);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : bfail(b, BOLTZ_EHIP, std::string("boltz_batch_set_step: ") + hipGetErrorString(e));
}

int boltz_batch_step(boltz_batch* b, const float* h_in, float* h_out, const boltz_walls* walls, void* stream) {
  if (!b) return BOLTZ_EINVAL;
  if (!h_in || !h_out) return bfail(b, BOLTZ_EINVAL, "boltz_batch_step: null buffer");
  if (overlap(h_in, h_out, (size_t)b->nodes * sizeof(float)))
    return bfail(b, BOLTZ_EINVAL, "boltz_batch_step: h_in and h_out overlap");
  if (b->any_cavity && !walls) return bfail(b, BOLTZ_EINVAL, "boltz_batch_step: cavities need walls");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // wall tables of every cavity (rebuilt only where the walls changed)
  for (int i = 0; i < b->count; ++i) {
    boltz_ctx* c = b->ctx[i];
    if (c->p.bc != BOLTZ_BC_CAVITY) continue;
    if (!walls_ok(&walls[i], c->p.nx))
      return bfail(b, BOLTZ_EINVAL, "boltz_batch_step: invalid walls of problem " + std::to_string(i));
    const int rc = ensure_ratio(c, make_walls(&walls[i]), &walls[i], st);
    if (rc != BOLTZ_OK) return bfail(b, rc, "boltz_batch_step: " + c->err);
  }
  auto ranged = [](int total) { return (total + 7) / 8; };
  if (b->total[0] > 0) {
    const int px = ranged(b->total[0]);
    hipLaunchKernelGGL(wall_batch_kernel<0>, dim3(8 * px), dim3(kWallBlock), 0, st, b->cavs, b->start[0], b->count,
                       h_in, px);
  }
  if (b->total[1] > 0) {
    const int px = ranged(b->total[1]);
    hipLaunchKernelGGL(wall_batch_kernel<1>, dim3(8 * px), dim3(kWallBlock), 0, st, b->cavs, b->start[1], b->count,
                       h_in, px);
  }
  if (b->stile == 0) {
    const int px = ranged(b->total[2]);
    if (b->order == 2)
      hipLaunchKernelGGL((stream4_batch_kernel<2, kTX4, kTY4>), dim3(8 * px), dim3(kTX4 * (kJ4 / 4)), 0, st, b->cavs,
                         b->start[2], b->count, h_in, h_out, px);
    else
      hipLaunchKernelGGL((stream4_batch_kernel<1, kTX4, kTY4>), dim3(8 * px), dim3(kTX4 * (kJ4 / 4)), 0, st, b->cavs,
                         b->start[2], b->count, h_in, h_out, px);
  } else {
    const int px = ranged(b->total_b);
    if (b->order == 2)
      hipLaunchKernelGGL((stream4_batch_kernel<2, kTX4b, kTY4b>), dim3(8 * px), dim3(kTX4b * (kJ4 / 4)), 0, st,
                         b->cavs, b->start_b, b->count, h_in, h_out, px);
    else
      hipLaunchKernelGGL((stream4_batch_kernel<1, kTX4b, kTY4b>), dim3(8 * px), dim3(kTX4b * (kJ4 / 4)), 0, st,
                         b->cavs, b->start_b, b->count, h_in, h_out, px);
  }
  if (b->total[3] > 0)
    hipLaunchKernelGGL(sample_batch_kernel, dim3(b->total[3]), dim3(kSampleBlock), b->sample_lds, st, b->cavs,
                       b->start[3], b->count, b->step_dev);
  if (b->total[4] > 0)
    hipLaunchKernelGGL(split_sort_batch_kernel, dim3(b->total[4]), dim3(kSortBlock), 0, st, b->cavs, b->start[4],
                       b->count);
  for (const BatchClass& K : b->cls) launch_class(b, K, h_out, h_out, st);
  hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, st, b->step_dev);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BOLTZ_OK : bfail(b, BOLTZ_EHIP, std::string("boltz_batch_step: ") + hipGetErrorString(e));
}

int boltz_batch_set_block(boltz_batch* b, int block) {
  if (!b) return BOLTZ_EINVAL;
  if (block != 256 && block != 512 && block != 1024)
    return bfail(b, BOLTZ_EINVAL, "boltz_batch_set_block: block size must be 256, 512 or 1024");
  bool any = false;
  for (const BatchClass& K : b->cls) any = any || K.ok[block_index(block)];
  if (!any) return bfail(b, BOLTZ_EINVAL, "boltz_batch_set_block: block size not available for any class");
  for (BatchClass& K : b->cls)
    if (K.ok[block_index(block)]) K.block = block;
  return BOLTZ_OK;
}

int boltz_batch_class_info(const boltz_batch* b, int index, boltz_batch_class* out) {
  if (!b || !out || index < 0 || index >= (int)b->cls.size()) return BOLTZ_EINVAL;
  const BatchClass& K = b->cls[index];
  for (int a = 0; a < 3; ++a) out->nv[a] = K.nv3[a];
  out->problems = K.problems;
  out->cells = K.cells;
  out->pair_cells = K.pair_cells;
  out->collide_block = K.block;
  out->pairs_per_lane = K.pu;
  out->spread = K.spread;
  out->grid = class_grid(K);
  out->cells_per_group = (K.nitems + out->grid - 1) / out->grid;
  out->ms = K.ms;
  return BOLTZ_OK;
}

int boltz_batch_set_class(boltz_batch* b, int index, int block, int pairs_per_lane, int spread) {
  if (!b) return BOLTZ_EINVAL;
  if (index < 0 || index >= (int)b->cls.size())
    return bfail(b, BOLTZ_EINVAL, "boltz_batch_set_class: no such class");
  BatchClass& K = b->cls[index];
  if ((block != 256 && block != 512 && block != 1024) || !K.ok[block_index(block)])
    return bfail(b, BOLTZ_EINVAL, "boltz_batch_set_class: block size not available for this class");
  if ((pairs_per_lane != 2 && pairs_per_lane != 4) || spread < 0 || spread > (K.part ? 1 : 2))
    return bfail(b, BOLTZ_EINVAL,
                 "boltz_batch_set_class: pairs_per_lane must be 2 or 4 and spread 0, 1 or 2 (0 or 1 for the "
                 "partial-tile layout)");
  K.block = block;
  K.pu = pairs_per_lane;
  K.spread = spread;
  return BOLTZ_OK;
}

int boltz_batch_set_stream_tile(boltz_batch* b, int tx, int ty) {
  if (!b) return BOLTZ_EINVAL;
  if (tx == kTX4 && ty == kTY4) b->stile = 0;
  else if (tx == kTX4b && ty == kTY4b) b->stile = 1;
  else return bfail(b, BOLTZ_EINVAL, "boltz_batch_set_stream_tile: tiles are 16 x 8 or 32 x 4 cells");
  return BOLTZ_OK;
}

int boltz_batch_tune(boltz_batch* b, float* h_a, float* h_b, const boltz_walls* walls, int steps, void* stream,
                     double* ms_out) {
  if (!b) return BOLTZ_EINVAL;
  if (!h_a || !h_b || steps < 1) return bfail(b, BOLTZ_EINVAL, "boltz_batch_tune: need two buffers and steps >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) return bfail(b, BOLTZ_EHIP, std::string("boltz_batch_tune: ") + hipGetErrorString(he));
  int rc = BOLTZ_OK;
  // milliseconds per call of f over `steps` calls after one warm-up call
  auto timed = [&](auto&& f, double& ms) {
    rc = f(0);
    if (rc != BOLTZ_OK) return false;
    (void)hipEventRecord(e0, st);
    for (int k = 0; k < steps && rc == BOLTZ_OK; ++k) rc = f(k + 1);
    (void)hipEventRecord(e1, st);
    he = hipEventSynchronize(e1);
    float t = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    if (he != hipSuccess) {
      rc = bfail(b, BOLTZ_EHIP, std::string("boltz_batch_tune: ") + hipGetErrorString(he));
      return false;
    }
    ms = (double)t / steps;
    return rc == BOLTZ_OK;
  };
  auto whole = [&](int k) { return boltz_batch_step(b, (k & 1) ? h_a : h_b, (k & 1) ? h_b : h_a, walls, stream); };
  double before = 0.0, after = 0.0;
  // 1. the stream tile shape, by whole steps
  bool ok = timed(whole, before);
  double best_ms = before;
  const int tile0 = b->stile;
  int best_tile = tile0;
  for (int t = 0; t < 2 && ok; ++t) {
    if (t == tile0) continue;
    b->stile = t;
    double ms = 0.0;
    ok = timed(whole, ms);
    if (ok && ms < best_ms) {
      best_ms = ms;
      best_tile = t;
    }
  }
  b->stile = best_tile;
  // 2. per class: block size x records per lane x workgroups, by the
  // class's collision launch alone (h_b -> h_a, the same input every time)
  const int blocks[3] = {256, 512, 1024};
  for (BatchClass& K : b->cls) {
    if (!ok) break;
    const BatchClass keep = K;
    BatchClass best = K;
    best.ms = 0.0;
    for (int t = 0; t < 3 && ok; ++t) {
      if (!K.ok[t]) continue;
      for (int pu = 2; pu <= 4 && ok; pu += 2)
        for (int sp = 0; sp < 3 && ok; ++sp) {
          K = keep;
          K.block = blocks[t];
          K.pu = pu;
          K.spread = sp;
          if (K.part && sp == 2) continue;
          double ms = 0.0;
          ok = timed(
              [&](int) {
                launch_class(b, K, h_b, h_a, st);
                const hipError_t le = hipGetLastError();
                return le == hipSuccess ? BOLTZ_OK
                                        : bfail(b, BOLTZ_EHIP, std::string("boltz_batch_tune: ") + hipGetErrorString(le));
              },
              ms);
          if (ok && (best.ms == 0.0 || ms < best.ms)) {
            best = K;
            best.ms = ms;
          }
        }
    }
    K = ok ? best : keep;
  }
  if (ok) ok = timed(whole, after);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms_out && ok) {
    ms_out[0] = before;
    ms_out[1] = after;
  }
  return rc;
}

}  // extern "C"
