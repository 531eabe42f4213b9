// C ABI of the unrolled solver: plane plan with checkpointing, forward and
// backward drivers.
//
// Iterations are grouped in segments of C = ckpt_every iterations.  The
// forward pass keeps, for every segment start s > 0, a checkpoint
// (f^s, f^{s-1}, p^s), and leaves the states of the last segment in the
// segment buffer.  The backward pass walks the segments from last to first;
// it recomputes a segment's states from its checkpoint (except for the last
// one) and then runs the adjoint steps of the segment in reverse.
//
// Where the states of segment j = [s, e) live (plane ids):
//   f^{s-1}, f^s : checkpoint j (segment 0: the g plane for both)
//   f^{e-1}      : the f^{s-1} slot of checkpoint j+1 when e < K
//   f^e          : the f^s slot of checkpoint j+1, or the output plane
//   f^k, p^k     : segment buffer slot k - s otherwise
//   p^s          : checkpoint j (segment 0: the zero planes)
//   p^e          : checkpoint j+1, or a discard slot when e = K
// so no state is ever copied.
#include <algorithm>
#include <atomic>
#include <cmath>

#include "unrolled.h"

namespace tvpd {
namespace {

// 2D adjoint steps as one fused pass (default) or as the two-pass reference.
std::atomic<int> g_fused_adjoint{1};

struct UPlan {
  int ndim, K, C, ncp;
  int G, Z, OUT, DUMP, CK0, SBF, SBP, A, B, T, PN, GBAR;
  int nplanes;

  int ckf(int j) const { return CK0 + (j - 1) * (2 + ndim); }
  int ckfm(int j) const { return ckf(j) + 1; }
  int ckp(int j) const { return ckf(j) + 2; }

  int f_slot(int j, int k) const {
    const int s = j * C, e = std::min(s + C, K);
    if (k == s - 1) return j == 0 ? G : ckfm(j);
    if (k == s) return j == 0 ? G : ckf(j);
    if (k == e - 1 && e < K && e - 1 > s) return ckfm(j + 1);
    if (k == e) return e < K ? ckf(j + 1) : OUT;
    return SBF + (k - s - 1);
  }
  int p_slot(int j, int k) const {
    const int s = j * C, e = std::min(s + C, K);
    if (k == s) return j == 0 ? Z : ckp(j);
    if (k == e) return e < K ? ckp(j + 1) : DUMP;
    return SBP + (k - s - 1) * ndim;
  }
};

UPlan make_plan(int ndim, int K, int ckpt) {
  UPlan p;
  p.ndim = ndim;
  p.K = K;
  p.C = std::max(1, std::min(ckpt, K));
  p.ncp = (K + p.C - 1) / p.C;
  int id = 0;
  p.G = id++;
  p.Z = id;
  id += ndim;
  p.OUT = id++;
  p.DUMP = id;
  id += ndim;
  p.CK0 = id;
  id += (p.ncp - 1) * (2 + ndim);
  p.SBF = id;
  id += std::max(p.C - 1, 0);
  p.SBP = id;
  id += std::max(p.C - 1, 0) * ndim;
  p.A = id;
  id += 2;
  p.B = id;
  id += 2;
  p.T = id;
  id += 2 * ndim;
  p.PN = id;
  id += ndim;
  p.GBAR = id++;
  p.nplanes = id;
  return p;
}

struct ULayout {
  UPlan plan;
  PlaneSet ps;       // base filled in later
  int64_t max_partials;
  size_t off_part, off_planes, bytes;
};

bool ushape_ok(const tvpd_shape* s, int batch) {
  if (!s || batch < 1) return false;
  if (s->ndim == 2) {
    if (s->nz != 1) return false;
  } else if (s->ndim != 3 || s->nz < 1) {
    return false;
  }
  return s->ny >= 1 && s->nx >= 1 && s->nx <= (1 << 20) && s->ny <= (1 << 20) &&
         s->nz <= (1 << 20);
}

int uargs_ok(const tvpd_shape* s, int batch, int K, int ckpt) {
  if (!ushape_ok(s, batch)) return TVPD_ERR_SHAPE;
  if (K < 1 || ckpt < 1) return TVPD_ERR_INVALID_ARG;
  // a segment of one iteration cannot hold f^{s-1} and f^s apart
  if (K > 1 && std::min(ckpt, K) < 2) return TVPD_ERR_INVALID_ARG;
  return TVPD_OK;
}

ULayout make_ulayout(const tvpd_shape& s, int batch, int K, int ckpt) {
  ULayout L;
  L.plan = make_plan(s.ndim, K, ckpt);
  PlaneSet& P = L.ps;
  P.base = nullptr;
  P.nb = batch;
  P.ndim = s.ndim;
  P.nz = s.nz;
  P.ny = s.ny;
  P.nx = s.nx;
  P.pitch = (int)round_up(s.nx, kColsPerLane);
  P.plane = round_up((int64_t)s.nz * s.ny * P.pitch, 64);
  P.istride = P.plane * L.plan.nplanes;
  L.max_partials = u_partials_needed(P);
  L.off_part = kHeaderBytes;
  L.off_planes = (size_t)round_up(L.off_part + L.max_partials * 8, kAlign);
  L.bytes = L.off_planes + (size_t)batch * P.istride * sizeof(float);
  return L;
}

int uws_ok(const ULayout& L, void* ws, size_t bytes) {
  if (!ws) return TVPD_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return TVPD_ERR_ALIGNMENT;
  if (bytes < L.bytes) return TVPD_ERR_WORKSPACE;
  return TVPD_OK;
}

#define UHIP(call)                                 \
  do {                                             \
    if ((call) != hipSuccess) return TVPD_ERR_HIP; \
  } while (0)

// Forward iterations k_from .. k_to-1 of segment j.  2D: passes of up to
// min(pass depth, 5) iterations, each iterate stored to its slot (the slots
// a pass writes are never among those it reads); 3D: one launch each.
int run_steps(const UPlan& p, const PlaneSet& P, int j, int k_from, int k_to,
              const float* coeffs, float theta, hipStream_t s) {
  if (P.ndim == 2) {
    const int depth = std::max(1, std::min(walk_depth(), kMaxPass - 1));
    for (int k = k_from; k < k_to;) {
      const int n = std::min(depth, k_to - k);
      PassIds ids;
      ids.fk = p.f_slot(j, k);
      ids.fkm = p.f_slot(j, k - 1);
      ids.pk = p.p_slot(j, k);
      for (int i = 0; i < kMaxPass; ++i) ids.fn[i] = ids.pn[i] = 0;
      for (int i = 1; i <= n; ++i) {
        ids.fn[i - 1] = p.f_slot(j, k + i);
        ids.pn[i - 1] = p.p_slot(j, k + i);
      }
      UHIP(launch_u_pass2d(P, ids, coeffs, k, n, theta, s));
      k += n;
    }
    return TVPD_OK;
  }
  for (int k = k_from; k < k_to; ++k) {
    StepIds ids;
    ids.fk = p.f_slot(j, k);
    ids.fkm = p.f_slot(j, k - 1);
    ids.pk = p.p_slot(j, k);
    ids.fn = p.f_slot(j, k + 1);
    ids.pn = p.p_slot(j, k + 1);
    UHIP(launch_u_step(P, ids, coeffs, k, theta, s));
  }
  return TVPD_OK;
}

}  // namespace

bool fused_adjoint_enabled() { return g_fused_adjoint.load() != 0; }

}  // namespace tvpd

using namespace tvpd;

extern "C" {

int tvpd_unrolled_workspace_size(const tvpd_shape* shape, int32_t batch,
                                 int32_t K, int32_t ckpt_every,
                                 size_t* bytes) {
  if (!bytes) return TVPD_ERR_INVALID_ARG;
  if (int rc = uargs_ok(shape, batch, K, ckpt_every)) return rc;
  *bytes = make_ulayout(*shape, batch, K, ckpt_every).bytes;
  return TVPD_OK;
}

int tvpd_unrolled_forward(const tvpd_shape* shape, int32_t batch,
                          const float* g, const float* coeffs, int32_t K,
                          int32_t ckpt_every, float theta, float* f_out,
                          void* ws, size_t ws_bytes, void* stream) {
  if (int rc = uargs_ok(shape, batch, K, ckpt_every)) return rc;
  if (!g || !coeffs || !f_out) return TVPD_ERR_INVALID_ARG;
  if (!(theta >= 0.0f && theta <= 1.0f)) return TVPD_ERR_INVALID_ARG;
  ULayout L = make_ulayout(*shape, batch, K, ckpt_every);
  if (int rc = uws_ok(L, ws, ws_bytes)) return rc;
  hipStream_t s = (hipStream_t)stream;
  PlaneSet P = L.ps;
  P.base = reinterpret_cast<float*>(static_cast<char*>(ws) + L.off_planes);
  const UPlan& p = L.plan;
  UHIP(launch_u_init(P, g, p.G, p.Z, p.ndim, s));
  for (int j = 0; j < p.ncp; ++j) {
    const int st = j * p.C, e = std::min(st + p.C, p.K);
    if (int rc = run_steps(p, P, j, st, e, coeffs, theta, s)) return rc;
  }
  UHIP(launch_u_read(P, p.OUT, f_out, s));
  return TVPD_OK;
}

int tvpd_unrolled_backward(const tvpd_shape* shape, int32_t batch,
                           const float* coeffs, int32_t K, int32_t ckpt_every,
                           float theta, const float* grad_f, float* grad_g,
                           float* grad_coeffs, void* ws, size_t ws_bytes,
                           void* stream) {
  if (int rc = uargs_ok(shape, batch, K, ckpt_every)) return rc;
  if (!coeffs || !grad_f || !grad_g || !grad_coeffs) return TVPD_ERR_INVALID_ARG;
  if (!(theta >= 0.0f && theta <= 1.0f)) return TVPD_ERR_INVALID_ARG;
  ULayout L = make_ulayout(*shape, batch, K, ckpt_every);
  if (int rc = uws_ok(L, ws, ws_bytes)) return rc;
  hipStream_t s = (hipStream_t)stream;
  PlaneSet P = L.ps;
  P.base = reinterpret_cast<float*>(static_cast<char*>(ws) + L.off_planes);
  double* partials =
      reinterpret_cast<double*>(static_cast<char*>(ws) + L.off_part);
  const UPlan& p = L.plan;
  // adjoint state: a = dL/df^K, b = 0, r = 0, gbar = 0
  UHIP(launch_u_zero(P, p.A, 2 + 2 + 2 * p.ndim + p.ndim + 1, s));
  UHIP(launch_u_load(P, grad_f, p.A, s));
  int ph = 0;
  for (int j = p.ncp - 1; j >= 0; --j) {
    const int st = j * p.C, e = std::min(st + p.C, p.K);
    if (j < p.ncp - 1) {
      if (int rc = run_steps(p, P, j, st, e - 1, coeffs, theta, s)) return rc;
    }
    for (int k = e - 1; k >= st; --k) {
      AdjIds a;
      a.fk = p.f_slot(j, k);
      a.fkm = p.f_slot(j, k - 1);
      a.pk = p.p_slot(j, k);
      a.g = p.G;
      a.a_in = p.A + ph;
      a.b_in = p.B + ph;
      a.r_in = p.T + ph * p.ndim;
      a.a_out = p.A + (ph ^ 1);
      a.b_out = p.B + (ph ^ 1);
      a.t_out = p.T + (ph ^ 1) * p.ndim;
      a.pn = p.PN;
      a.gbar = p.GBAR;
      UHIP(launch_u_adjoint(P, a, coeffs, k, theta, partials, L.max_partials,
                            grad_coeffs, s));
      ph ^= 1;
    }
  }
  UHIP(launch_u_final_grad(P, p.GBAR, p.A + ph, p.B + ph, grad_g, s));
  return TVPD_OK;
}

int tvpd_set_fused_adjoint(int32_t on) {
  if (on != 0 && on != 1) return TVPD_ERR_INVALID_ARG;
  g_fused_adjoint.store(on);
  return TVPD_OK;
}

}  // extern "C"
