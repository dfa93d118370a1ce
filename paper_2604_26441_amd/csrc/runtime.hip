// C ABI of libsimpgmg: hierarchy setup, operator application, V-cycle and
// PCG orchestration on one HIP stream.  All arithmetic runs in the kernels of
// this library; host code only sequences launches and reads back scalars.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "batch.hpp"
#include "bstage.hpp"
#include "kernels.hpp"
#include "unet.hpp"

namespace sgmg {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

// Device scalar slots.
enum Slot {
  SC_FF = 0, SC_RR0 = 1,     // pcg init: f.f, r.r (adjacent: one 2-sum)
  SC_PQ = 2, SC_RR = 3,
  SC_RZ0 = 4, SC_ROZ0 = 5,   // r.z, r_old.z for even iterations (adjacent)
  SC_RZ1 = 6, SC_ROZ1 = 7,   // odd iterations
  SC_TRUE = 8,               // true residual norm^2
  SC_XW = 9, SC_XDX = 10, SC_NRM = 11, SC_DSUM = 12, SC_EPS = 13, SC_MAX = 14,
  SC_SEQ = 15,               // count of PCG iterations run on this hierarchy
  SC_COUNT = 16
};

struct Level {
  Grid g{};
  bool f32 = false;          // work vectors of this level are float
  uint8_t* fixn = nullptr;
  double* d64 = nullptr;
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  double* S64 = nullptr;     // l >= 1
  float* S32 = nullptr;      // l >= 1 when stored in FP32
  double lam = 0.0;          // raw power-iteration estimate
  int n_free = 0;
  void* b = nullptr;         // work vectors (T = float or double)
  void* x[2] = {nullptr, nullptr};
  void* dv = nullptr;
  void* r = nullptr;
};

}  // namespace sgmg

using namespace sgmg;

struct sgmg_hierarchy {
  sgmg_options o{};
  int L = 0;
  Level lev[8];
  KeTables kt{};
  std::vector<void*> allocs;
  double* ke64 = nullptr;
  float* ke32 = nullptr;
  double* gtab = nullptr;
  double* E64 = nullptr;
  float* E32 = nullptr;
  float* E32s = nullptr;     // E / s for the MFMA kernel
  // MFMA launch shape [nsplit == 3]: element rows per wave tile, node planes
  // per wave (tuned per mesh, or the default)
  int mfma_rows[3] = {4, 4, 1};     // [BF16, BF16X3, FP64]; FP64 rows 0: node kernel,
  int mfma_zchunk[3] = {4, 4, 4};   // rows 1: sum/difference-basis tiles
  uint16_t* atab = nullptr;  // MFMA A-operand table (BF16 bits)
  double* atab64 = nullptr;  // FP64 MFMA A-operand table
  // level 1 without its stored stencil (FP64 level 1 above the coarsest):
  // the child moduli of each coarse element, the elements and nodes the
  // product leaves to the stencil, and the list of those nodes
  double* l1_E8 = nullptr;
  uint8_t* l1_el = nullptr;
  uint8_t* l1_skip = nullptr;
  int* l1_list = nullptr;
  int l1_nlist = 0;
  double* l1_Sd = nullptr;   // their stencil rows, gathered entry-major
  bool l1_mf = false;        // level-1 applies use it (else the stencil)
  int l1_zchunk = 2;         // its node planes per wave tile
  double maxE_lambda = 0.0;  // max E when lambdas were estimated
  int nL = 0;
  int* free_idx = nullptr;
  double* Ainv = nullptr;
  double* Apack = nullptr;   // upper-triangle tiles of Ainv (the per-cycle operand)
  double* symv_part = nullptr;
  double coarse_eps = 0.0;
  bool coarse_iter = false;  // coarsest solve: fixed-count PCG instead of the dense inverse
  double* cpcg_p = nullptr;  // its second search direction and z (2 n), per-step partials, flags
  double* cpcg_scratch = nullptr;
  int* cpcg_done = nullptr;
  RedWs ws{};
  size_t npart = 0;          // doubles in ws.partials
  // the PCG's r.z fused into the V-cycle's last fine smoothing step (BF16-
  // family MFMA operator): the dot partner, set while an iteration graph is
  // recorded, and that kernel's block partials (size: its largest grid)
  const double* vc_dot64 = nullptr;
  double* rz_part = nullptr;
  size_t n_rz_part = 0;
  double* sc = nullptr;
  double* h_sc = nullptr;    // pinned mirror of sc
  double* h_it = nullptr;    // coherent, device-mapped: the scalars of the last PCG
                             // iteration of each slot parity (2 x SC_COUNT), then
                             // the iteration counter's last value
  double* d_it = nullptr;    // device address of h_it
  int* d_flag = nullptr;
  double* r = nullptr;
  double* z = nullptr;
  double* p = nullptr;
  double* q = nullptr;
  double* r_old = nullptr;
  double* tmp = nullptr;
  double* xs = nullptr;      // solver-owned copy of the iterate (graphs bind it)
  double* xs2 = nullptr;     // second iterate buffer: a PCG iteration of slot parity
                             // p reads x from one buffer and writes the other, so
                             // the previous iterate survives a queued successor
  // flexible GMRES: basis V (kry_cols + 1 columns), Z (kry_cols columns) and
  // small device arrays for the Hessenberg column and y; sized on first use
  double* kry = nullptr;
  double* kry_small = nullptr;
  int kry_cols = 0;
  double* gj_scratch = nullptr;
  hipStream_t cap = nullptr; // capture stream
  // per preconditioner: the iteration graphs of the two slot parities and the
  // graph of the solve prologue (z_0 = M r_0, r_0.z_0, p_0 = z_0)
  hipGraphExec_t iter_graph[3][3] = {};
};

namespace {

constexpr size_t kMinPartials = 1 << 16;

// Process-wide autotuning results: (nx, ny, nz, variant) -> MFMA launch shape
// (rows, z-chunk); variant 1 = BF16, 3 = BF16X3, 64 = FP64.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tune;

std::pair<int, int> tuned_shape(int nx, int ny, int nz, int variant, std::pair<int, int> dflt) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(nx, ny, nz, variant));
  return it == g_tune.end() ? dflt : it->second;
}

int dalloc(sgmg_hierarchy* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
    *p = nullptr;
    return SGMG_ENOMEM;
  }
  h->allocs.push_back(*p);
  return 0;
}

template <typename T>
int dalloc_t(sgmg_hierarchy* h, T** p, size_t count) {
  void* v = nullptr;
  int rc = dalloc(h, &v, count * sizeof(T));
  *p = (T*)v;
  return rc;
}

#define TRY(x)                 \
  do {                         \
    int _rc = (x);             \
    if (_rc) return _rc;       \
  } while (0)

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("kernel launch: ") + hipGetErrorString(e));
    return SGMG_EHIP;
  }
  return 0;
}

// Local prolongation of pattern p (px + 3 py + 9 pz): rows fine local DOFs,
// columns coarse local DOFs (see the device table of the same name).
const double kPat[3][2][2] = {{{1.0, 0.0}, {0.5, 0.5}}, {{0.5, 0.5}, {0.0, 1.0}},
                              {{0.0, 1.0}, {0.0, 1.0}}};

void build_gtab(const KeTables& kt, std::vector<double>& g) {
  g.assign(27 * 576, 0.0);
  for (int p = 0; p < 27; ++p) {
    const int px = p % 3, py = (p / 3) % 3, pz = p / 9;
    double P[24][24] = {};
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) {
        const double w = kPat[px][a & 1][b & 1] * kPat[py][(a >> 1) & 1][(b >> 1) & 1] *
                         kPat[pz][a >> 2][b >> 2];
        for (int c = 0; c < 3; ++c) P[3 * a + c][3 * b + c] = w;
      }
    // G = P^T K P
    double KP[24][24];
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) {
        double s = 0.0;
        for (int k = 0; k < 24; ++k) s += kt.ke[i * 24 + k] * P[k][j];
        KP[i][j] = s;
      }
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) {
        double s = 0.0;
        for (int k = 0; k < 24; ++k) s += P[k][i] * KP[k][j];
        g[(size_t)p * 576 + i * 24 + j] = s;
      }
  }
}

template <typename T>
Epi<T> epi_store(T* out, RedWs ws = {}, double* dot_out = nullptr) {
  Epi<T> e{};
  e.mode = EPI_STORE;
  e.out = out;
  e.want_dot = dot_out != nullptr;
  e.ws = ws;
  e.dot_out = dot_out;
  return e;
}

// STORE with the x.y block partials left in ws.partials (no finalize).
template <typename T>
Epi<T> epi_store_partials(T* out, RedWs ws) {
  Epi<T> e = epi_store<T>(out, ws);
  e.want_dot = 1;
  return e;
}

template <typename T>
Epi<T> epi_resid(T* out, const T* b) {
  Epi<T> e{};
  e.mode = EPI_RESID;
  e.out = out;
  e.b = b;
  return e;
}

template <typename T>
Epi<T> epi_smooth(T* xout, const T* b, const T* dinv, T* d, double c1, double c2, int store_d,
                  double* out64) {
  Epi<T> e{};
  e.mode = EPI_SMOOTH;
  e.out = xout;
  e.b = b;
  e.dinv = dinv;
  e.d = d;
  e.c1 = c1;
  e.c2 = c2;
  e.store_d = store_d;
  e.out64 = out64;
  return e;
}

// y-side operator application on level l in the level's own precision.
template <typename T>
int apply_level(const sgmg_hierarchy* h, int l, sgmg_prec prec, const T* x, const Epi<T>& ep,
                hipStream_t s);

template <>
int apply_level<double>(const sgmg_hierarchy* h, int l, sgmg_prec prec, const double* x,
                        const Epi<double>& ep, hipStream_t s) {
  const Level& L = h->lev[l];
  if (prec != SGMG_F64) {
    set_error("double vectors require SGMG_F64");
    return SGMG_EINVAL;
  }
  if (l == 0 && h->mfma_rows[2] == 1 && sf64_size_ok(L.g)) {
    launch_apply_fine_sf64(L.g, h->mfma_zchunk[2], h->E64, h->kt.lam, h->kt.mu, x, L.fixn, ep, s);
  } else if (l == 0 && h->mfma_rows[2] > 1 && mfma64_size_ok(L.g)) {
    launch_apply_fine_mfma64(L.g, h->mfma_rows[2], h->mfma_zchunk[2], h->E64, h->atab64, x, L.fixn,
                             ep, s);
  } else if (l == 0) {
    launch_apply_fine_node<double>(L.g, h->E64, h->ke64, x, L.fixn, ep, s);
  } else if (l == 1 && h->l1_mf && !ep.want_dot) {
    // rows next to Dirichlet DOFs (or odd-axis ends) from the stencil, the
    // rest from the element products, in one launch
    launch_apply_l1_haar(L.g, h->l1_zchunk, h->l1_E8, h->kt.lam, h->kt.mu, x, L.fixn, h->l1_skip,
                         h->l1_Sd, h->l1_list, h->l1_nlist, ep, s);
  } else {
    launch_stencil_apply<double>(L.g, L.S64, x, L.fixn, ep,
                                 h->o.stencil_form == 3 ? 0 : h->o.stencil_form, s);
  }
  return check_launch();
}

template <>
int apply_level<float>(const sgmg_hierarchy* h, int l, sgmg_prec prec, const float* x,
                       const Epi<float>& ep, hipStream_t s) {
  const Level& L = h->lev[l];
  if (l == 0) {
    if (prec == SGMG_F32) {
      launch_apply_fine_node<float>(L.g, h->E32, h->ke32, x, L.fixn, ep, s);
    } else if (prec == SGMG_BF16 || prec == SGMG_BF16X3 || prec == SGMG_BF16X2) {
      if (!h->kt.integral) {
        set_error("BF16 MFMA path needs s*K_e integral (nu = 0.3 family); use F32");
        return SGMG_EINVAL;
      }
      if (!mfma_size_ok(L.g)) {
        set_error("BF16 MFMA path: level-0 vector of 2^30 bytes or more; use F32");
        return SGMG_EINVAL;
      }
      const int ns = prec == SGMG_BF16 ? 1 : prec == SGMG_BF16X2 ? 2 : 3;
      launch_apply_fine_mfma(L.g, ns, h->mfma_rows[ns >= 2], h->mfma_zchunk[ns >= 2], h->E32s,
                             h->atab, x, L.fixn, ep, s);
    } else {
      set_error("float vectors need F32, BF16 or BF16X3");
      return SGMG_EINVAL;
    }
  } else {
    if (!L.S32 || prec != SGMG_F32) {
      set_error("level is not stored in FP32");
      return SGMG_EINVAL;
    }
    launch_stencil_apply<float>(L.g, L.S32, x, L.fixn, ep,
                                h->o.stencil_form == 3 ? 0 : h->o.stencil_form, s);
  }
  return check_launch();
}

// Block partials that the level-0 FP64 operator writes with a dot (its grid
// size: the MFMA tile grid or one block per 256 nodes).
int k64_dot_partials(const sgmg_hierarchy* h) {
  const Level& L = h->lev[0];
  if (h->mfma_rows[2] == 1 && sf64_size_ok(L.g))
    return (int)apply_fine_sf64_blocks(L.g, h->mfma_zchunk[2]);
  if (h->mfma_rows[2] > 1 && mfma64_size_ok(L.g))
    return (int)apply_fine_mfma_blocks(L.g, h->mfma_rows[2] == 4 ? 4 : 8,
                                       h->mfma_zchunk[2] < 1 ? 1 : h->mfma_zchunk[2]);
  return div_up(L.g.Nn, 256);
}

sgmg_prec level_prec(const sgmg_hierarchy* h, int l) {
  if (l == 0) return h->o.fine_prec;
  if (l == 1 && l < h->L - 1) return h->o.level1_prec;
  return SGMG_F64;
}

// ---------------------------------------------------------------------------
// Power iteration for lambda_max(D^-1 K^l) in FP64 (Sec. 3.5).
int power_lambda(sgmg_hierarchy* h, int l, int iters, hipStream_t s, double* out) {
  Level& L = h->lev[l];
  const int n = L.g.n;
  double* x = h->p;
  double* w = h->q;
  double* y = h->z;
  launch_power_start(x, L.fixn, L.g.Nn, h->o.seed + (uint64_t)l, s);
  launch_dot(x, nullptr, nullptr, n, h->ws, h->sc + SC_NRM, s);
  launch_normalize(x, h->sc + SC_NRM, x, n, s);
  for (int k = 0; k < iters; ++k) {
    TRY(apply_level<double>(h, l, SGMG_F64, x, epi_store<double>(w, h->ws, h->sc + SC_XW), s));
    if (k == iters - 1) {
      launch_dot(x, x, L.d64, n, h->ws, h->sc + SC_XDX, s);
    } else {
      launch_scale_dinv_norm(L.dinv64, w, y, n, h->ws, h->sc + SC_NRM, s);
      launch_normalize(y, h->sc + SC_NRM, x, n, s);
    }
  }
  TRY(check_launch());
  SGMG_HIP(hipMemcpyAsync(h->h_sc, h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  SGMG_HIP(hipStreamSynchronize(s));
  double lam = iters > 0 ? h->h_sc[SC_XW] / h->h_sc[SC_XDX] : 0.0;
  if (!(lam > 1e-6) || !std::isfinite(lam)) lam = 1e-6;
  *out = lam;
  return 0;
}

// All E-dependent parts: moduli, diagonals, Galerkin operators, coarsest inverse.
int assemble_operators(sgmg_hierarchy* h, const double* rho_or_E, hipStream_t s) {
  const sgmg_options& o = h->o;
  Level& L0 = h->lev[0];
  launch_simp(rho_or_E, h->E64, h->E32, L0.g.nel, o.input_is_modulus, o.E0, o.Emin, o.penal, s);
  launch_scale_E(h->E64, h->E32s, L0.g.nel, 1.0 / h->kt.kscale, s);
  launch_diag_fine(L0.g, h->E64, h->ke64, L0.fixn, L0.d64, s);
  for (int l = 1; l < h->L; ++l) {
    Level& F = h->lev[l - 1];
    Level& C = h->lev[l];
    if (l == 1)
      launch_galerkin_l1(F.g, C.g, h->E64, h->gtab, h->ke64, F.fixn, C.fixn, C.S64, s);
    else
      launch_galerkin_stencil(F.g, C.g, F.S64, C.fixn, C.S64, s);
    launch_stencil_diag(C.g, C.S64, C.d64, s);
    if (C.S32) launch_stencil_to_f32(C.S64, C.S32, (size_t)kStencil * C.g.Nn, s);
  }
  if (h->l1_E8)
    launch_l1_child_moduli(L0.g, h->lev[1].g, h->E64, L0.fixn, h->l1_E8, h->l1_el, s);
  if (h->l1_Sd)
    launch_stencil_gather_rows<double>(h->lev[1].g, h->lev[1].S64, h->l1_list, h->l1_nlist,
                                       h->l1_Sd, s);
  TRY(check_launch());
  // D^-1 with the floor max(D, 1e-30 max D) on free DOFs, 0 on fixed DOFs.
  for (int l = 0; l < h->L; ++l) {
    Level& L = h->lev[l];
    launch_max_nonneg(L.d64, L.fixn, L.g.n, h->sc + SC_MAX, s);
    launch_diag_finalize(L.d64, L.dinv64, L.dinv32, L.fixn, L.g.n, h->sc + SC_MAX, s);
  }
  TRY(check_launch());
  // coarsest: dense K_L + eps I and its explicit inverse
  Level& C = h->lev[h->L - 1];
  const int nf = h->nL;
  if (nf > 0 && !h->coarse_iter) {
    launch_dense_assemble(C.g, C.S64, h->free_idx, nf, h->Ainv, s);
    launch_dense_diag_sum(h->Ainv, nf, h->ws, h->sc + SC_DSUM, s);
    launch_dense_add_diag(h->Ainv, nf, h->sc + SC_DSUM, s, h->sc + SC_EPS);
    SGMG_HIP(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
    dense_spd_inverse(h->Ainv, nf, h->gj_scratch, h->d_flag, s);
    TRY(check_launch());
    int flag = 0;
    SGMG_HIP(hipMemcpyAsync(&flag, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipMemcpyAsync(h->h_sc, h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipStreamSynchronize(s));
    h->coarse_eps = h->h_sc[SC_EPS];
    if (flag) {
      set_error("coarsest factorisation met a non-positive pivot");
      return SGMG_EFACTOR;
    }
    launch_dense_pack(h->Ainv, nf, h->Apack, s);
    TRY(check_launch());
  }
  return 0;
}

double max_modulus(sgmg_hierarchy* h, hipStream_t s) {
  launch_max_nonneg(h->E64, nullptr, h->lev[0].g.nel, h->sc + SC_MAX, s);
  double m = 0.0;
  if (hipMemcpyAsync(&m, h->sc + SC_MAX, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return 0.0;
  return m;
}

int estimate_lambdas(sgmg_hierarchy* h, hipStream_t s) {
  for (int l = 0; l < h->L - 1; ++l) {
    if (h->o.lambda_override) {
      h->lev[l].lam = h->o.lambda_override[l];
      continue;
    }
    const int it = l == 0 ? h->o.power_iters_fine : h->o.power_iters_coarse;
    TRY(power_lambda(h, l, it, s, &h->lev[l].lam));
  }
  h->maxE_lambda = max_modulus(h, s);
  return 0;
}

// ---------------------------------------------------------------------------
// V-cycle (Eq. vcycle).  On entry lev[l].b holds the right-hand side and
// lev[l].x[0] the first smoothing step from zero (written by the producer).
// On exit lev[l].x[*cur] holds V^l(b).
struct Smoother {
  bool cheb;
  int steps;
  double omega, theta, delta, sigma1;
};

// Whether the first smoothing step from zero (fused into the PCG update or
// the cycle entry) must also write its direction d = x_1 for the second
// step: only when that step stores a direction of its own into d (more than
// two Chebyshev steps); with two the second step reads x_1 in place of d.
bool entry_writes_d(const Smoother& sm) { return sm.cheb && sm.steps > 2; }

Smoother smoother_of(const sgmg_hierarchy* h, int l) {
  Smoother sm{};
  const double lam = h->o.lambda_safety * h->lev[l].lam;
  sm.cheb = (l == 0 && h->o.fine_smoother == 0);
  sm.steps = l == 0 ? h->o.fine_degree : h->o.coarse_sweeps;
  sm.omega = std::min(h->o.jacobi_omega_max, 4.0 / (3.0 * lam));
  sm.theta = 0.5 * lam * (1.0 + h->o.cheb_alpha);
  sm.delta = 0.5 * lam * (1.0 - h->o.cheb_alpha);
  sm.sigma1 = sm.theta / sm.delta;
  return sm;
}

double first_step_coef(const Smoother& sm) { return sm.cheb ? 1.0 / sm.theta : sm.omega; }

int vcycle_level(const sgmg_hierarchy* h, int l, int* cur, double* out64, bool from_zero,
                 hipStream_t s);

template <typename TF, typename TC>
int descend(const sgmg_hierarchy* h, int l, const TF* r, hipStream_t s) {
  const Level& F = h->lev[l];
  const Level& C = h->lev[l + 1];
  if (l + 1 == h->L - 1) {
    launch_restrict<TF, TC>(F.g, C.g, r, C.fixn, (TC*)C.b, nullptr, 0.0, nullptr, nullptr, s);
  } else {
    const Smoother cs = smoother_of(h, l + 1);
    const TC* dinv = std::is_same<TC, float>::value ? (const TC*)C.dinv32 : (const TC*)C.dinv64;
    launch_restrict<TF, TC>(F.g, C.g, r, C.fixn, (TC*)C.b, dinv, first_step_coef(cs),
                            (TC*)C.x[0], cs.cheb ? (TC*)C.dv : nullptr, s);
  }
  return check_launch();
}

template <typename T>
int smooth_and_recurse(const sgmg_hierarchy* h, int l, int* cur, double* out64, bool from_zero,
                       hipStream_t s) {
  const Level& L = h->lev[l];
  const Smoother sm = smoother_of(h, l);
  const sgmg_prec prec = level_prec(h, l);
  const T* b = (const T*)L.b;
  const T* dinv = std::is_same<T, float>::value ? (const T*)L.dinv32 : (const T*)L.dinv64;
  T* d = (T*)L.dv;
  // From zero, x[0] already holds the first pre-smoothing step (fused into
  // the restriction or the cycle entry); otherwise pre-smoothing starts from
  // the iterate in x[*cur] and takes all its steps here.
  int c = from_zero ? 0 : *cur;
  double rho = sm.cheb ? 1.0 / sm.sigma1 : 0.0;
  for (int k = from_zero ? 1 : 0; k < sm.steps; ++k) {
    double c1 = 0.0, c2 = sm.omega;
    if (sm.cheb) {
      if (k == 0) {
        c2 = 1.0 / sm.theta;
      } else {
        const double rn = 1.0 / (2.0 * sm.sigma1 - rho);
        c1 = rn * rho;
        c2 = 2.0 * rn / sm.delta;
        rho = rn;
      }
    }
    // the pass's last direction is never read again (the next pass starts
    // with c1 = 0), so it is not stored
    const int store_d = sm.cheb && k < sm.steps - 1;
    // the second step from zero reads its direction d = x_1 - 0 from x_1
    // itself when nothing stores a direction there (entry_writes_d)
    T* dk = (from_zero && k == 1 && !entry_writes_d(sm)) ? (T*)L.x[c] : d;
    TRY(apply_level<T>(h, l, prec, (const T*)L.x[c],
                       epi_smooth<T>((T*)L.x[1 - c], b, dinv, dk, c1, c2, store_d, nullptr), s));
    c = 1 - c;
  }
  // residual, restriction, coarse correction
  TRY(apply_level<T>(h, l, prec, (const T*)L.x[c], epi_resid<T>((T*)L.r, b), s));
  const Level& C = h->lev[l + 1];
  if (C.f32) TRY((descend<T, float>(h, l, (const T*)L.r, s)));
  else TRY((descend<T, double>(h, l, (const T*)L.r, s)));
  int cc = 0;
  TRY(vcycle_level(h, l + 1, &cc, nullptr, true, s));
  // W-cycle: a second coarse cycle from the first one's result, unless the
  // coarser level is the coarsest (solved exactly once)
  for (int g = 1; g < h->o.cycle_gamma && l + 2 < h->L; ++g)
    TRY(vcycle_level(h, l + 1, &cc, nullptr, false, s));
  if (C.f32) launch_prolong_add<T, float>(L.g, C.g, (const float*)C.x[cc], L.fixn, (T*)L.x[c], s);
  else launch_prolong_add<T, double>(L.g, C.g, (const double*)C.x[cc], L.fixn, (T*)L.x[c], s);
  TRY(check_launch());
  // post-smoothing from the corrected iterate
  rho = sm.cheb ? 1.0 / sm.sigma1 : 0.0;
  for (int k = 0; k < sm.steps; ++k) {
    double c1 = 0.0, c2 = sm.omega;
    if (sm.cheb) {
      if (k == 0) {
        c2 = 1.0 / sm.theta;
      } else {
        const double rn = 1.0 / (2.0 * sm.sigma1 - rho);
        c1 = rn * rho;
        c2 = 2.0 * rn / sm.delta;
        rho = rn;
      }
    }
    const bool last = k == sm.steps - 1;
    double* o64 = last ? out64 : nullptr;
    // the cycle's result leaves through out64 only: the level's own copy of
    // the last iterate is not written
    T* xout = last && out64 ? nullptr : (T*)L.x[1 - c];
    Epi<T> e = epi_smooth<T>(xout, b, dinv, d, c1, c2, sm.cheb && !last, o64);
    if (l == 0 && last && out64 && h->vc_dot64) {
      // the PCG's r.z: block partials of r . out64 (see pcg_body)
      e.dot64 = h->vc_dot64;
      e.ws.partials = h->rz_part;
    }
    TRY(apply_level<T>(h, l, prec, (const T*)L.x[c], e, s));
    c = 1 - c;
  }
  *cur = c;
  return 0;
}

// One cycle on level l for the right-hand side in lev[l].b.  from_zero: the
// iterate starts at zero (its first smoothing step is already in x[0]);
// otherwise it starts from x[*cur].  The result is left in x[*cur].
int vcycle_level(const sgmg_hierarchy* h, int l, int* cur, double* out64, bool from_zero,
                 hipStream_t s) {
  const Level& L = h->lev[l];
  if (l == h->L - 1) {
    if (h->coarse_iter)
      launch_coarse_pcg(L.g, L.S64, L.dinv64, L.fixn, (const double*)L.b, (double*)L.x[0],
                        (double*)L.r, h->cpcg_p + L.g.n, (double*)L.dv, h->cpcg_p, (double*)L.x[1],
                        h->cpcg_scratch,
                        h->cpcg_done, h->o.coarse_pcg_iters, s);
    else
      launch_dense_symv(h->Apack, h->free_idx, h->nL, (const double*)L.b, h->symv_part,
                        (double*)L.x[0], s);
    *cur = 0;
    return check_launch();
  }
  if (L.f32) return smooth_and_recurse<float>(h, l, cur, out64, from_zero, s);
  return smooth_and_recurse<double>(h, l, cur, out64, from_zero, s);
}

int vcycle_full(const sgmg_hierarchy* h, const double* r, double* z, hipStream_t s) {
  const Level& L = h->lev[0];
  const Smoother sm = smoother_of(h, 0);
  const double c0 = first_step_coef(sm);
  if (L.f32)
    launch_vcycle_entry<float>(r, (float*)L.b, L.dinv32, c0, (float*)L.x[0],
                               entry_writes_d(sm) ? (float*)L.dv : nullptr, L.g.n, s);
  else
    launch_vcycle_entry<double>(r, (double*)L.b, L.dinv64, c0, (double*)L.x[0],
                                entry_writes_d(sm) ? (double*)L.dv : nullptr, L.g.n, s);
  TRY(check_launch());
  int cur = 0;
  return vcycle_level(h, 0, &cur, z, true, s);
}

int validate(const sgmg_options* o) {
  if (!o) { set_error("options is NULL"); return SGMG_EINVAL; }
  // every hierarchy has at least two levels, so each axis must coarsen once
  if (o->nx < 2 || o->ny < 2 || o->nz < 2) { set_error("mesh dims must be >= 2"); return SGMG_EINVAL; }
  if ((long)(o->nx + 1) * (o->ny + 1) * (o->nz + 1) * 3 > 0x7fffffffL) {
    set_error("mesh too large for 32-bit DOF indexing");
    return SGMG_EINVAL;
  }
  if (o->n_levels == 1 || o->n_levels < 0 || o->n_levels > 8) {
    set_error("n_levels must be 0 (auto) or 2..8");
    return SGMG_EINVAL;
  }
  if (o->fine_degree < 1 || o->coarse_sweeps < 1) { set_error("smoothing steps must be >= 1"); return SGMG_EINVAL; }
  if (o->fine_prec < SGMG_F64 || o->fine_prec > SGMG_BF16X2) { set_error("bad fine_prec"); return SGMG_EINVAL; }
  if (o->level1_prec != SGMG_F64 && o->level1_prec != SGMG_F32) { set_error("level1_prec must be F64 or F32"); return SGMG_EINVAL; }
  if (!(o->cheb_alpha > 0.0 && o->cheb_alpha < 1.0)) { set_error("cheb_alpha must be in (0,1)"); return SGMG_EINVAL; }
  if (!(o->lambda_safety > 0.0)) { set_error("lambda_safety must be > 0"); return SGMG_EINVAL; }
  if (o->cycle_gamma != 1 && o->cycle_gamma != 2) { set_error("cycle_gamma must be 1 or 2"); return SGMG_EINVAL; }
  if (o->stencil_form < 0 || o->stencil_form > 3) { set_error("stencil_form must be 0, 1, 2 or 3"); return SGMG_EINVAL; }
  if (o->bf16_guard && (o->guard_window < 1 || !(o->guard_drop >= 1.0))) {
    set_error("bf16_guard needs guard_window >= 1 and guard_drop >= 1");
    return SGMG_EINVAL;
  }
  return 0;
}

}  // namespace

// ===========================================================================
namespace sgmg {
int hierarchy_fine_view(const ::sgmg_hierarchy* h, FineView* v) {
  if (!h || !v) return SGMG_EINVAL;
  v->g = h->lev[0].g;
  v->fixn = h->lev[0].fixn;
  v->ke = h->ke64;
  v->is_modulus = h->o.input_is_modulus;
  v->E0 = h->o.E0;
  v->Emin = h->o.Emin;
  v->penal = h->o.penal;
  return 0;
}
}  // namespace sgmg

extern "C" {

const char* sgmg_last_error(void) { return g_err.c_str(); }

static int capture_vcycle_graphs(sgmg_hierarchy* h, hipStream_t s);

void sgmg_default_options(sgmg_options* o, int nx, int ny, int nz) {
  std::memset(o, 0, sizeof(*o));
  o->nx = nx; o->ny = ny; o->nz = nz;
  o->nu = 0.3; o->E0 = 1.0; o->Emin = 1e-9; o->penal = 3.0;
  o->input_is_modulus = 0;
  o->n_levels = 4;
  o->fine_smoother = 0;
  o->fine_degree = 2;
  o->coarse_sweeps = 2;
  o->cheb_alpha = 1.0 / 30.0;
  o->jacobi_omega_max = 0.5;
  o->lambda_safety = 1.3;
  o->power_iters_fine = 20;
  o->power_iters_coarse = 10;
  o->fine_prec = SGMG_F32;
  o->level1_prec = SGMG_F64;
  o->dense_max = 5000;
  o->coarse_pcg_iters = 80;
  o->seed = 0;
  o->flexible_beta = 0;
  o->stag_window = 0;
  o->lambda_override = nullptr;
  o->use_graphs = 1;
  o->cycle_gamma = 1;
  o->stencil_form = 0;
  o->bf16_guard = 1;
  o->guard_window = 50;
  o->guard_drop = 10.0;
}

void sgmg_destroy(sgmg_hierarchy* h) {
  if (!h) return;
  for (auto& row : h->iter_graph)
    for (auto& g : row)
      if (g) hipGraphExecDestroy(g);
  if (h->cap) hipStreamDestroy(h->cap);
  for (void* p : h->allocs) hipFree(p);
  if (h->kry) hipFree(h->kry);
  if (h->kry_small) hipFree(h->kry_small);
  if (h->h_sc) hipHostFree(h->h_sc);
  if (h->h_it) hipHostFree(h->h_it);
  delete h;
}

int sgmg_setup_hierarchy(const sgmg_options* opts, const double* rho_or_E, const uint8_t* fixed_dof,
                         void* stream, sgmg_hierarchy** out) {
  if (out) *out = nullptr;
  TRY(validate(opts));
  if (!rho_or_E || !out) { set_error("NULL argument"); return SGMG_EINVAL; }
  hipStream_t s = as_stream(stream);
  sgmg_hierarchy* h = new (std::nothrow) sgmg_hierarchy();
  if (!h) { set_error("host allocation failed"); return SGMG_ENOMEM; }
  h->o = *opts;
  h->o.lambda_override = nullptr;
  int rc = 0;
  auto fail = [&](int code) { sgmg_destroy(h); return code; };

  compute_ke(opts->nu, &h->kt);
  for (int q = 0; q < 3; ++q) {
    // FP64 defaults to the vector-ALU sum/difference-basis tiles (rows 1, 4
    // planes) until tuned
    const auto sh = tuned_shape(opts->nx, opts->ny, opts->nz, q == 2 ? 64 : (q ? 3 : 1),
                                q == 2 ? std::make_pair(1, 4) : std::make_pair(4, 4));
    h->mfma_rows[q] = sh.first;
    h->mfma_zchunk[q] = sh.second;
  }
  // level dims by floor coarsening and masks by injection
  Grid g0 = make_grid(opts->nx, opts->ny, opts->nz);
  int maxL = opts->n_levels ? opts->n_levels : 8;
  std::vector<Grid> grids{g0};
  for (int l = 1; l < maxL; ++l) {
    const Grid& f = grids.back();
    if (f.nx / 2 < 1 || f.ny / 2 < 1 || f.nz / 2 < 1) break;
    grids.push_back(make_grid(f.nx / 2, f.ny / 2, f.nz / 2));
  }
  if ((int)grids.size() < std::max(2, opts->n_levels)) {
    set_error("mesh cannot be coarsened to the requested number of levels");
    return fail(SGMG_EINVAL);
  }
  // masks on the device, free counts on the host
  std::vector<uint8_t*> masks;
  for (size_t l = 0; l < grids.size(); ++l) {
    uint8_t* m = nullptr;
    if ((rc = dalloc_t(h, &m, grids[l].Nn))) return fail(rc);
    masks.push_back(m);
  }
  if (fixed_dof) launch_mask_from_dofs(fixed_dof, masks[0], g0.Nn, s);
  else launch_mask_cantilever(g0, masks[0], s);
  for (size_t l = 1; l < grids.size(); ++l)
    launch_mask_inject(grids[l - 1], grids[l], masks[l - 1], masks[l], s);
  if ((rc = check_launch())) return fail(rc);
  std::vector<int> nfree(grids.size());
  for (size_t l = 0; l < grids.size(); ++l) {
    std::vector<uint8_t> fx(grids[l].Nn);
    if (hipMemcpyAsync(fx.data(), masks[l], grids[l].Nn, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("mask download failed");
      return fail(SGMG_EHIP);
    }
    int c = 0;
    for (uint8_t v : fx) c += 3 - __builtin_popcount(v & 7);
    nfree[l] = c;
  }
  int L = opts->n_levels;
  if (!L) {
    L = (int)grids.size();
    for (int k = 2; k <= (int)grids.size(); ++k)
      if (nfree[k - 1] <= opts->dense_max) { L = k; break; }
  }
  // Above the dense cutoff the coarsest solve is fixed-count PCG (Sec. 3.2).
  h->coarse_iter = nfree[L - 1] > opts->dense_max;
  if (h->coarse_iter && opts->coarse_pcg_iters < 1) {
    set_error("coarsest level has " + std::to_string(nfree[L - 1]) +
              " free DOFs, more than dense_max, and coarse_pcg_iters < 1");
    return fail(SGMG_EINVAL);
  }
  h->L = L;
  h->o.n_levels = L;
  size_t maxn = 0;
  for (int l = 0; l < L; ++l) {
    Level& V = h->lev[l];
    V.g = grids[l];
    V.fixn = masks[l];
    V.n_free = nfree[l];
    const sgmg_prec p = level_prec(h, l);
    V.f32 = (l < L - 1) && p != SGMG_F64;
    const size_t n = V.g.n;
    maxn = std::max(maxn, n);
    if ((rc = dalloc_t(h, &V.d64, n)) || (rc = dalloc_t(h, &V.dinv64, n)) ||
        (rc = dalloc_t(h, &V.dinv32, n)))
      return fail(rc);
    if (l >= 1) {
      if ((rc = dalloc_t(h, &V.S64, (size_t)kStencil * V.g.Nn))) return fail(rc);
      if (l == 1 && V.f32 && (rc = dalloc_t(h, &V.S32, (size_t)kStencil * V.g.Nn))) return fail(rc);
    }
    const size_t es = V.f32 ? sizeof(float) : sizeof(double);
    if ((rc = dalloc(h, &V.b, n * es)) || (rc = dalloc(h, &V.x[0], n * es)) ||
        (rc = dalloc(h, &V.x[1], n * es)) || (rc = dalloc(h, &V.dv, n * es)) ||
        (rc = dalloc(h, &V.r, n * es)))
      return fail(rc);
    hipMemsetAsync(V.x[0], 0, n * es, s);
    hipMemsetAsync(V.x[1], 0, n * es, s);
  }
  for (size_t l = L; l < masks.size(); ++l) { /* unused coarser masks stay allocated */ }
  // constants
  if ((rc = dalloc_t(h, &h->ke64, 576)) || (rc = dalloc_t(h, &h->ke32, 576)) ||
      (rc = dalloc_t(h, &h->gtab, 27 * 576)))
    return fail(rc);
  std::vector<double> gt;
  build_gtab(h->kt, gt);
  hipMemcpyAsync(h->ke64, h->kt.ke, 576 * sizeof(double), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(h->ke32, h->kt.ke32, 576 * sizeof(float), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(h->gtab, gt.data(), gt.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if ((rc = dalloc_t(h, &h->E64, g0.nel)) || (rc = dalloc_t(h, &h->E32, g0.nel)) ||
      (rc = dalloc_t(h, &h->E32s, g0.nel)) || (rc = dalloc_t(h, &h->atab, 2 * 64 * 8)) ||
      (rc = dalloc_t(h, &h->atab64, 2 * 6 * 64)))
    return fail(rc);
  {
    std::vector<uint16_t> at(2 * 64 * 8);
    build_mfma_atab(h->kt, at.data());
    hipMemcpyAsync(h->atab, at.data(), at.size() * sizeof(uint16_t), hipMemcpyHostToDevice, s);
    std::vector<double> at64(2 * 6 * 64);
    build_mfma_atab64(h->kt, at64.data());
    hipMemcpyAsync(h->atab64, at64.data(), at64.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (hipStreamSynchronize(s) != hipSuccess) { set_error("sync failed"); return fail(SGMG_EHIP); }
  }
  // reductions, scalars, PCG vectors
  // one partial per block of the largest reduction grid (fused dots run one
  // block per 256 nodes; vector reductions use at most 2 x 1024 slots)
  // (the MFMA kernel's largest grid is its smallest tile shape: 4 rows, 1 plane;
  // the FP64 sum-factorised kernel's tiles have the same geometry)
  // (+ 4096: the PCG iteration keeps the r.r partials after the K p ones)
  // (a Galerkin level's apply with a dot: at most three blocks per 64 nodes)
  const size_t npart = std::max({kMinPartials, (size_t)div_up(g0.Nn, 256) + 2048,
                                 apply_fine_mfma_blocks(g0, 4, 1) + 4096,
                                 h->L > 1 ? stencil_apply_blocks(h->lev[1].g) : (size_t)0});
  h->npart = npart;
  h->n_rz_part = apply_fine_mfma_blocks(g0, 4, 1);
  if ((rc = dalloc_t(h, &h->rz_part, h->n_rz_part))) return fail(rc);
  if ((rc = dalloc_t(h, &h->ws.partials, npart)) || (rc = dalloc_t(h, &h->ws.counter, 1)) ||
      (rc = dalloc_t(h, &h->sc, SC_COUNT)) || (rc = dalloc_t(h, &h->d_flag, 1)))
    return fail(rc);
  hipMemsetAsync(h->ws.counter, 0, sizeof(unsigned), s);
  hipMemsetAsync(h->sc, 0, SC_COUNT * sizeof(double), s);
  if (hipHostMalloc((void**)&h->h_it, (2 * SC_COUNT + 1) * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&h->d_it, h->h_it, 0) != hipSuccess) {
    set_error("pinned allocation failed");
    return fail(SGMG_ENOMEM);
  }  std::memset(h->h_it, 0, (2 * SC_COUNT + 1) * sizeof(double));

  if (hipHostMalloc((void**)&h->h_sc, SC_COUNT * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    set_error("pinned allocation failed");
    return fail(SGMG_ENOMEM);
  }
  for (double** v : {&h->r, &h->z, &h->p, &h->q, &h->r_old, &h->tmp, &h->xs, &h->xs2})
    if ((rc = dalloc_t(h, v, maxn))) return fail(rc);
  // coarsest free index list
  {
    Level& C = h->lev[L - 1];
    std::vector<uint8_t> fx(C.g.Nn);
    hipMemcpyAsync(fx.data(), C.fixn, C.g.Nn, hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) { set_error("sync failed"); return fail(SGMG_EHIP); }
    std::vector<int> idx;
    for (int i = 0; i < C.g.n; ++i)
      if (!((fx[i / 3] >> (i % 3)) & 1)) idx.push_back(i);
    h->nL = (int)idx.size();
    const size_t nd = h->coarse_iter ? 1 : (size_t)std::max(h->nL, 1);  // dense-solve sizes
    if ((rc = dalloc_t(h, &h->free_idx, std::max<size_t>(idx.size(), 1))) ||
        (rc = dalloc_t(h, &h->Ainv, nd * nd)) ||
        (rc = dalloc_t(h, &h->gj_scratch, nd * 64 + 64 * 64)))
      return fail(rc);
    const size_t nt = h->coarse_iter ? 1 : (size_t)std::max(sym_tiles(h->nL), 1);
    if ((rc = dalloc_t(h, &h->Apack, nt * 64 * 64)) ||
        (rc = dalloc_t(h, &h->symv_part, nt * 2 * 64)))
      return fail(rc);
    if (!idx.empty())
      hipMemcpyAsync(h->free_idx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, s);
  }
  if (h->coarse_iter) {
    const Grid& cg = h->lev[L - 1].g;
    const int it = opts->coarse_pcg_iters;
    if ((rc = dalloc_t(h, &h->cpcg_p, 2 * (size_t)cg.n)) ||
        (rc = dalloc_t(h, &h->cpcg_scratch, coarse_pcg_scratch(cg, it))) ||
        (rc = dalloc_t(h, &h->cpcg_done, (size_t)it + 1)))
      return fail(rc);
  }
  // level 1 without its stored stencil: FP64 level 1 above the coarsest
  const bool l1mf = L > 2 && !h->lev[1].f32 && (opts->stencil_form == 3 || opts->stencil_form == 0) &&
                    l1_haar_size_ok(h->lev[1].g);
  if (l1mf) {
    const Grid& c1 = h->lev[1].g;
    if ((rc = dalloc_t(h, &h->l1_E8, (size_t)c1.nel * 8)) ||
        (rc = dalloc_t(h, &h->l1_el, (size_t)c1.nel)) ||
        (rc = dalloc_t(h, &h->l1_skip, (size_t)c1.Nn)))
      return fail(rc);
  }
  if ((rc = assemble_operators(h, rho_or_E, s))) return fail(rc);
  if (l1mf) {
    // the nodes left to the stencil depend on the Dirichlet masks only
    const Grid& c1 = h->lev[1].g;
    launch_l1_skip_nodes(c1, h->l1_el, h->lev[1].fixn, h->l1_skip, s);
    if ((rc = check_launch())) return fail(rc);
    std::vector<uint8_t> sk((size_t)c1.Nn);
    if (hipMemcpyAsync(sk.data(), h->l1_skip, sk.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("level-1 node flags copy failed");
      return fail(SGMG_EHIP);
    }
    std::vector<int> list;
    for (int i = 0; i < c1.Nn; ++i)
      if (sk[i]) list.push_back(i);
    h->l1_nlist = (int)list.size();
    if ((rc = dalloc_t(h, &h->l1_list, std::max<size_t>(list.size(), 1))) ||
        (rc = dalloc_t(h, &h->l1_Sd, (size_t)kStencil * std::max<size_t>(list.size(), 1))))
      return fail(rc);
    if (!list.empty())
      hipMemcpyAsync(h->l1_list, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, s);
    launch_stencil_gather_rows<double>(c1, h->lev[1].S64, h->l1_list, h->l1_nlist, h->l1_Sd, s);
    if ((rc = check_launch())) return fail(rc);
    // form 3 asks for it; with form 0 the autotuner's choice for this mesh
    // (kept with the launch shapes, key 101), else the stencil
    h->l1_mf = opts->stencil_form == 3;
    const auto l1 = tuned_shape(opts->nx, opts->ny, opts->nz, 101, std::make_pair(-1, 0));
    if (l1.first >= 0) {
      if (opts->stencil_form == 0) h->l1_mf = l1.first == 1;
      if (l1.second > 0) h->l1_zchunk = l1.second;
    }
  }
  if (opts->lambda_override) h->o.lambda_override = opts->lambda_override;
  rc = estimate_lambdas(h, s);
  h->o.lambda_override = nullptr;
  if (rc) return fail(rc);
  if ((rc = capture_vcycle_graphs(h, s))) return fail(rc);
  if (hipStreamSynchronize(s) != hipSuccess) { set_error("sync failed"); return fail(SGMG_EHIP); }
  *out = h;
  return 0;
}

int sgmg_update_moduli(sgmg_hierarchy* h, const double* rho_or_E, void* stream) {
  if (!h || !rho_or_E) { set_error("NULL argument"); return SGMG_EINVAL; }
  hipStream_t s = as_stream(stream);
  TRY(assemble_operators(h, rho_or_E, s));
  const double m = max_modulus(h, s);
  if (h->maxE_lambda <= 0.0 || std::fabs(m - h->maxE_lambda) > 0.1 * h->maxE_lambda) {
    // new spectral estimates change the smoothing coefficients that the
    // iteration graphs hold; the operators themselves stay in place
    for (auto& row : h->iter_graph)
      for (auto& g : row)
        if (g) { hipGraphExecDestroy(g); g = nullptr; }
    TRY(estimate_lambdas(h, s));
  }
  TRY(capture_vcycle_graphs(h, s));
  SGMG_HIP(hipStreamSynchronize(s));
  return 0;
}

int sgmg_apply_K(const sgmg_hierarchy* h, int level, sgmg_prec prec, const void* u, void* y,
                 void* stream) {
  if (!h || !u || !y) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (level < 0 || level >= h->L) { set_error("level out of range"); return SGMG_EINVAL; }
  if (u == y) { set_error("u and y must not alias"); return SGMG_EINVAL; }
  hipStream_t s = as_stream(stream);
  if (prec == SGMG_F64)
    return apply_level<double>(h, level, prec, (const double*)u, epi_store<double>((double*)y), s);
  return apply_level<float>(h, level, prec, (const float*)u, epi_store<float>((float*)y), s);
}

int sgmg_vcycle(const sgmg_hierarchy* h, const double* r, double* z, void* stream) {
  if (!h || !r || !z) { set_error("NULL argument"); return SGMG_EINVAL; }
  return vcycle_full(h, r, z, as_stream(stream));
}

// Iterate buffers of a PCG iteration with rz slot `slot`: it reads x from
// *xin and writes *xout (parity 0 writes xs, parity 1 writes xs2).
static void pcg_iterates(const sgmg_hierarchy* h, int slot, double** xin, double** xout) {
  const bool even = slot == SC_RZ0;
  *xout = even ? h->xs : h->xs2;
  *xin = even ? h->xs2 : h->xs;
}

// One PCG iteration on device buffers only (so it can be captured):
// q = K p (p.q), x = x_prev + alpha p, r -= alpha q (r.r), z = M r, r.z (and
// r_old.z), p = z + beta p.  Scalars stay on the device in slot pairs and
// the iterate in buffers that alternate with the iteration parity.
static int pcg_body(sgmg_hierarchy* h, int precond, int slot, hipStream_t s) {
  const Level& L0 = h->lev[0];
  const int n = L0.g.n;
  double* sc = h->sc;
  double *xin, *xout;
  pcg_iterates(h, slot, &xin, &xout);
  const bool flex = h->o.flexible_beta != 0;
  const int nslot = slot == SC_RZ0 ? SC_RZ1 : SC_RZ0;
  // The r.r partials of the update and the r.z partials after the
  // preconditioner are summed inside the p update (no finalize launches);
  // they sit in disjoint parts of the workspace.
  // The K p partials (summed inside the update) come first; the r.r
  // partials of the update start after both them and the r.z partials.
  const int nb = pcg_vec_partials(n);
  const int npq = k64_dot_partials(h);
  RedWs ws_rr = h->ws;
  ws_rr.partials = h->ws.partials + std::max(2 * (size_t)nb, (size_t)npq);
  if (std::max(2 * (size_t)nb, (size_t)npq) + nb > h->npart) {
    set_error("reduction workspace too small");
    return SGMG_EINVAL;
  }
  TRY(apply_level<double>(h, 0, SGMG_F64, h->p, epi_store_partials<double>(h->q, h->ws), s));
  // With the V-cycle as preconditioner, a fixed beta and a BF16-family MFMA
  // fine level, the cycle's last smoothing step also forms r.z (the r.z
  // launch and its reading of r and z drop out)
  const sgmg_prec p0 = level_prec(h, 0);
  const bool fuse_rz = precond == 2 && !flex && h->L > 1 && L0.f32 && smoother_of(h, 0).steps >= 1 &&
                       (p0 == SGMG_BF16 || p0 == SGMG_BF16X3 || p0 == SGMG_BF16X2);
  int nrz = 0;
  if (fuse_rz) {
    const int ns = p0 == SGMG_BF16 ? 1 : p0 == SGMG_BF16X2 ? 2 : 3;
    const int rows = h->mfma_rows[ns >= 2] == 4 ? 4 : 8;
    nrz = (int)apply_fine_mfma_blocks(L0.g, rows, std::max(1, h->mfma_zchunk[ns >= 2]));
    if ((size_t)nrz > h->n_rz_part) {
      set_error("fused r.z partials exceed their workspace");
      return SGMG_EINVAL;
    }
  }
  if (precond == 2) {
    // the update also writes the V-cycle's entry (its first smoothing step)
    const Smoother sm = smoother_of(h, 0);
    const double c0 = first_step_coef(sm);
    if (L0.f32)
      launch_pcg_update_xr_entry<float>(xin, xout, h->r, flex ? h->r_old : nullptr, h->p, h->q,
                                        sc, slot, SC_PQ, h->ws.partials, npq, n, ws_rr, nullptr, (float*)L0.b,
                                        L0.dinv32, c0, (float*)L0.x[0],
                                        entry_writes_d(sm) ? (float*)L0.dv : nullptr, s);
    else
      launch_pcg_update_xr_entry<double>(xin, xout, h->r, flex ? h->r_old : nullptr, h->p, h->q,
                                         sc, slot, SC_PQ, h->ws.partials, npq, n, ws_rr, nullptr, (double*)L0.b,
                                         L0.dinv64, c0, (double*)L0.x[0],
                                         entry_writes_d(sm) ? (double*)L0.dv : nullptr, s);
    TRY(check_launch());
    int cur = 0;
    if (fuse_rz) h->vc_dot64 = h->r;
    const int rc = vcycle_level(h, 0, &cur, h->z, true, s);
    h->vc_dot64 = nullptr;
    TRY(rc);
  } else {
    launch_pcg_update_xr_entry<double>(xin, xout, h->r, flex ? h->r_old : nullptr, h->p, h->q,
                                       sc, slot, SC_PQ, h->ws.partials, npq, n, ws_rr, nullptr, nullptr, nullptr, 0.0,
                                       nullptr, nullptr, s);
    if (precond == 1) launch_apply_dinv(L0.dinv64, h->r, h->z, n, s);
    else launch_copy(h->r, h->z, n, s);
  }
  if (!fuse_rz) launch_pcg_dot_rz(h->r, h->z, flex ? h->r_old : nullptr, n, h->ws, nullptr, s);
  launch_pcg_update_p_red(h->p, h->z, fuse_rz ? h->rz_part : h->ws.partials,
                          fuse_rz ? nrz : nb, ws_rr.partials, sc, nslot, flex ? 1 : 0, slot, SC_RR,
                          SC_PQ, SC_SEQ, h->d_it + SC_COUNT * (slot == SC_RZ0 ? 0 : 1),
                          h->d_it + 2 * SC_COUNT, n, s);
  return check_launch();
}

// PCG prologue on the solver's own buffers: z = M r, r.z into sc[SC_RZ0],
// p = z.
static int pcg_prologue_body(sgmg_hierarchy* h, int precond, hipStream_t s) {
  const Level& L0 = h->lev[0];
  const int n = L0.g.n;
  if (precond == 2) TRY(vcycle_full(h, h->r, h->z, s));
  else if (precond == 1) launch_apply_dinv(L0.dinv64, h->r, h->z, n, s);
  else launch_copy(h->r, h->z, n, s);
  launch_pcg_dot_rz(h->r, h->z, nullptr, n, h->ws, h->sc + SC_RZ0, s);
  launch_copy(h->z, h->p, n, s);
  return check_launch();
}

// Captures (once) the graph of one PCG iteration for a preconditioner and
// slot parity (par 0, 1), or of the prologue (par 2).  Capture records the
// launches without running them.
static int ensure_graph(sgmg_hierarchy* h, int precond, int par, hipStream_t s) {
  const int slot = par == 0 ? SC_RZ0 : SC_RZ1;
  hipGraphExec_t& ge = h->iter_graph[precond][par];
  if (!ge) {
    if (!h->cap) SGMG_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    // the capture stream must not run ahead of work already queued on s
    SGMG_HIP(hipStreamSynchronize(s));
    SGMG_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    const int rc = par == 2 ? pcg_prologue_body(h, precond, h->cap)
                            : pcg_body(h, precond, slot, h->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &g);
    if (rc) { if (g) hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) { set_error(std::string("graph capture: ") + hipGetErrorString(e)); return SGMG_EHIP; }
    const hipError_t e2 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) { ge = nullptr; set_error(std::string("graph instantiate: ") + hipGetErrorString(e2)); return SGMG_EHIP; }
  }
  return 0;
}

// Whether the PCG loop may queue iteration it + 1 before reading back
// iteration it, given the relative residuals rel_0 .. rel_{it-1}: only when
// iteration it is predicted to stay above rtol by a wide margin (the last
// step ratio, at most 1/2, applied with a further factor 1/4), so that a
// discarded look-ahead iteration is rare.
static bool lookahead_ok(const std::vector<double>& hist, double rtol) {
  const size_t m = hist.size();
  if (m == 0) return false;
  double q = 0.5;
  if (m >= 2 && hist[m - 2] > 0.0) q = std::min(q, hist[m - 1] / hist[m - 2]);
  return hist[m - 1] * q * 0.25 >= rtol;
}

static int run_body(sgmg_hierarchy* h, int precond, int slot, hipStream_t s) {
  if (!h->o.use_graphs) return pcg_body(h, precond, slot, s);
  const int par = slot == SC_RZ0 ? 0 : 1;
  TRY(ensure_graph(h, precond, par, s));
  SGMG_HIP(hipGraphLaunch(h->iter_graph[precond][par], s));
  return 0;
}

static int run_prologue(sgmg_hierarchy* h, int precond, hipStream_t s) {
  if (!h->o.use_graphs) return pcg_prologue_body(h, precond, s);
  TRY(ensure_graph(h, precond, 2, s));
  SGMG_HIP(hipGraphLaunch(h->iter_graph[precond][2], s));
  return 0;
}

// The V-cycle-preconditioned iteration graphs are part of the hierarchy:
// captured at setup and after every re-assembly, so a solve only launches.
static int capture_vcycle_graphs(sgmg_hierarchy* h, hipStream_t s) {
  if (!h->o.use_graphs) return 0;
  TRY(ensure_graph(h, 2, 0, s));
  TRY(ensure_graph(h, 2, 1, s));
  return ensure_graph(h, 2, 2, s);
}

int sgmg_pcg_solve(sgmg_hierarchy* h, int precond, const double* f, double* u, double rtol,
                   int maxit, sgmg_solve_info* info, void* stream) {
  if (!h || !f || !u) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (precond < 0 || precond > 2 || maxit < 0) { set_error("bad precond or maxit"); return SGMG_EINVAL; }
  hipStream_t s = as_stream(stream);
  const Level& L0 = h->lev[0];
  const int n = L0.g.n;
  double* sc = h->sc;
  double* hs = h->h_sc;
  hipEvent_t e0, e1;
  SGMG_HIP(hipEventCreate(&e0));
  SGMG_HIP(hipEventCreate(&e1));
  SGMG_HIP(hipEventRecord(e0, s));
  auto K64 = [&](const double* x, double* y, double* dot_out) {
    return apply_level<double>(h, 0, SGMG_F64, x, epi_store<double>(y, h->ws, dot_out), s);
  };
  auto precondition = [&](const double* r, double* z) -> int {
    if (precond == 2) return vcycle_full(h, r, z, s);
    if (precond == 1) launch_apply_dinv(L0.dinv64, r, z, n, s);
    else launch_copy(r, z, n, s);
    return check_launch();
  };
  auto readsc = [&]() -> int {
    SGMG_HIP(hipMemcpyAsync(hs, sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipStreamSynchronize(s));
    return 0;
  };
  int status = SGMG_MAXIT, iters = 0;
  double rel = 0.0, rel_true = -1.0, nf = 0.0;
  std::vector<double> hist;
  int rc = 0;
  // x_0 lives in xs2, where the first iteration (slot SC_RZ0) reads it
  double* xcur = h->xs2;
  // The iteration of slot parity q writes its scalars to h_it + q SC_COUNT
  // from its last kernel, then the hierarchy's iteration count to
  // h_it[2 SC_COUNT].  The host waits for the count that the launch will
  // write (no event between iteration graphs); while waiting it checks now
  // and then that the stream still has work, so a failed launch cannot leave
  // it spinning.
  auto par = [](int sl) { return sl == SC_RZ0 ? 0 : 1; };
  double seq_next = 0.0;             // count the next iteration launch writes
  double seq_of[2] = {0.0, 0.0};     // count awaited per parity
  const volatile double* seq_host = h->h_it + 2 * SC_COUNT;
  auto launch_iter = [&](int sl) -> int {
    TRY(run_body(h, precond, sl, s));
    seq_of[par(sl)] = seq_next;
    seq_next += 1.0;
    return 0;
  };
  auto wait_iter = [&](int sl) -> int {
    const double target = seq_of[par(sl)];
    for (unsigned k = 1; *seq_host < target; ++k) {
      if ((k & 4095) == 0) {
        const hipError_t q = hipStreamQuery(s);
        if (q == hipSuccess && *seq_host < target) {
          set_error("PCG iteration scalars did not arrive");
          return SGMG_EHIP;
        }
        if (q != hipSuccess && q != hipErrorNotReady) {
          set_error(std::string("PCG iteration: ") + hipGetErrorString(q));
          return SGMG_EHIP;
        }
      }
      __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return 0;
  };
  // Guarded BF16 (Sec. 3.5, 3.6): on a failed step, a non-positive or
  // non-finite r.z, or too little progress over guard_window iterations, the
  // level-0 smoothing switches to the FP32-accurate BF16X3 split and the
  // recurrence restarts (beta = 0) from the current iterate and its FP64
  // true residual.  The captured V-cycle graphs hold the BF16 kernels, so
  // they are dropped (and captured again when next launched).
  const bool guard = h->o.bf16_guard && precond == 2 && h->o.fine_prec == SGMG_BF16;
  int fallback_it = -1;
  auto drop_graphs = [&]() -> int {
    SGMG_HIP(hipStreamSynchronize(s));
    for (auto& g : h->iter_graph[2])
      if (g) { hipGraphExecDestroy(g); g = nullptr; }
    return 0;
  };
  auto fallback = [&](int it, int nslot, double& rz) -> int {
    TRY(drop_graphs());
    h->o.fine_prec = SGMG_BF16X3;
    fallback_it = it;
    TRY(K64(xcur, h->tmp, nullptr));
    launch_residual(f, h->tmp, h->tmp, n, h->ws, sc + SC_TRUE, s);
    launch_copy(h->tmp, h->r, n, s);
    TRY(precondition(h->r, h->z));
    launch_pcg_dot_rz(h->r, h->z, nullptr, n, h->ws, sc + nslot, s);
    launch_copy(h->z, h->p, n, s);
    TRY(readsc());
    rz = hs[nslot];
    rel = std::sqrt(hs[SC_TRUE]) / nf;
    return 0;
  };
  hipEvent_t e_pro = nullptr;
  SGMG_HIP(hipEventCreateWithFlags(&e_pro, hipEventDisableTiming));
  launch_copy(u, xcur, n, s);
  do {
    // Prologue: r_0 = f - K x_0, z_0 = M r_0, p_0 = z_0 and their scalars are
    // queued together with iteration 1 (which writes only the other iterate
    // buffer) before the host reads the scalars, so an early exit below
    // leaves x_0 intact and merely discards that iteration.
    if ((rc = K64(xcur, h->q, nullptr))) break;
    launch_pcg_init(f, h->q, 1, h->r, n, h->ws, sc + SC_FF, s);
    if ((rc = run_prologue(h, precond, s))) break;
    SGMG_HIP(hipMemcpyAsync(hs, sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipEventRecord(e_pro, s));
    // (the copy above is ordered before iteration 1, so hs[SC_SEQ] is the
    // count before this solve's first iteration)
    bool queued = false;    // iteration `it` is already on the stream
    int slot = SC_RZ0;
    if (maxit > 0) {
      if ((rc = launch_iter(slot))) break;
      queued = true;
    }
    SGMG_HIP(hipEventSynchronize(e_pro));
    seq_of[0] += hs[SC_SEQ] + 1.0;
    seq_next += hs[SC_SEQ] + 1.0;
    nf = std::sqrt(hs[SC_FF]);
    if (nf == 0.0) {
      SGMG_HIP(hipMemsetAsync(xcur, 0, n * sizeof(double), s));
      status = SGMG_CONVERGED; rel = 0.0; rel_true = 0.0;
      hist.push_back(0.0);
      break;
    }
    rel = std::sqrt(hs[SC_RR0]) / nf;
    hist.push_back(rel);
    if (!std::isfinite(rel)) { status = SGMG_NONFINITE; break; }
    if (rel < rtol) { status = SGMG_CONVERGED; rel_true = rel; break; }
    if (maxit == 0) { status = SGMG_MAXIT; break; }
    if (!std::isfinite(hs[SC_RZ0])) { status = SGMG_NONFINITE; break; }
    if (hs[SC_RZ0] <= 0.0) { status = SGMG_BREAKDOWN; break; }
    // Look-ahead: iteration it + 1 is queued before the scalars of iteration
    // it are read back whenever the residual history says that iteration it
    // will not stop the solve, so the device does not idle while the host
    // decides.  Iteration it + 1 reads only device state and writes the
    // other iterate buffer, so if iteration it does stop the solve (a
    // misprediction) x_it is intact and the queued iteration is discarded;
    // the iterates and scalars are those of the plain loop either way.
    for (int it = 1; it <= maxit; ++it) {
      const int nslot = slot == SC_RZ0 ? SC_RZ1 : SC_RZ0;
      if (!queued && (rc = launch_iter(slot))) break;
      queued = false;
      if (it < maxit && lookahead_ok(hist, rtol)) {
        if ((rc = launch_iter(nslot))) break;
        queued = true;
      }
      if ((rc = wait_iter(slot))) break;
      const volatile double* hi = h->h_it + SC_COUNT * par(slot);
      double* xin;
      pcg_iterates(h, slot, &xin, &xcur);     // a failed step copies x_{it-1} here
      const double pq = hi[SC_PQ];
      const bool can_fall = guard && fallback_it < 0;
      // a failed step leaves x_it = x_{it-1} (the update kernel skips it)
      const bool step_failed = !std::isfinite(pq) || pq <= 0.0;
      if (step_failed && !can_fall) {
        status = std::isfinite(pq) ? SGMG_BREAKDOWN : SGMG_NONFINITE;
        iters = it - 1;
        break;
      }
      iters = it;
      double rz = hi[nslot];
      if (!step_failed) rel = std::sqrt(hi[SC_RR]) / nf;
      if (!step_failed && !std::isfinite(rel) && !can_fall) {
        hist.push_back(rel);
        status = SGMG_NONFINITE;
        break;
      }
      if (!step_failed && rel < rtol) {
        // (queued after a look-ahead iteration, which touches neither x_it
        // nor tmp)
        if ((rc = K64(xcur, h->tmp, nullptr))) break;
        launch_residual(f, h->tmp, h->tmp, n, h->ws, sc + SC_TRUE, s);
        if ((rc = readsc())) break;
        const double rt = std::sqrt(hs[SC_TRUE]) / nf;
        if (rt < rtol) { hist.push_back(rel); status = SGMG_CONVERGED; rel_true = rt; break; }
        // residual replacement with a restart of the recurrence (beta = 0);
        // it rebuilds r, z, p and r.z from x_it, so a look-ahead iteration
        // is dropped and run again from the new state
        launch_copy(h->tmp, h->r, n, s);
        if ((rc = precondition(h->r, h->z))) break;
        launch_pcg_dot_rz(h->r, h->z, nullptr, n, h->ws, sc + nslot, s);
        launch_copy(h->z, h->p, n, s);
        if ((rc = readsc())) break;
        queued = false;
        rz = hs[nslot];
        rel = rt;
      }
      if (can_fall) {
        bool trip = step_failed || !std::isfinite(rel) || !std::isfinite(rz) || rz <= 0.0;
        const int gw = h->o.guard_window;
        if (!trip && it >= gw) trip = !(rel * h->o.guard_drop <= hist[it - gw]);
        if (trip) {
          if ((rc = fallback(it, nslot, rz))) break;
          queued = false;
        }
      }
      hist.push_back(rel);
      const int w = h->o.stag_window;
      if (w > 0 && it >= w) {
        const double recent = *std::min_element(hist.end() - w, hist.end());
        const double before = *std::min_element(hist.begin(), hist.end() - w);
        if (recent > 0.99 * before) { status = SGMG_STAGNATED; break; }
      }
      if (it == maxit) { status = SGMG_MAXIT; break; }
      if (!std::isfinite(rz)) { status = SGMG_NONFINITE; break; }
      if (rz <= 0.0) { status = SGMG_BREAKDOWN; break; }
      slot = nslot;
    }
  } while (0);
  hipEventDestroy(e_pro);
  if (fallback_it >= 0) {            // the hierarchy is BF16 again for later calls
    const int rc2 = drop_graphs();
    h->o.fine_prec = SGMG_BF16;
    if (!rc) rc = rc2;
  }
  if (rc) {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
  }
  launch_copy(xcur, u, n, s);
  SGMG_HIP(hipEventRecord(e1, s));
  if (rel_true < 0.0) {
    TRY(K64(xcur, h->tmp, nullptr));
    launch_residual(f, h->tmp, nullptr, n, h->ws, sc + SC_TRUE, s);
    TRY(readsc());
    rel_true = std::sqrt(hs[SC_TRUE]) / (nf > 0 ? nf : 1.0);
  }
  SGMG_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (info) {
    info->status = status;
    info->iters = iters;
    info->rel_res_true = rel_true;
    info->rel_res_recur = rel;
    info->solve_ms = ms;
    info->fallback_iter = fallback_it;
    if (info->history && info->history_cap > 0) {
      const int m = std::min<int>(info->history_cap, (int)hist.size());
      for (int i = 0; i < m; ++i) info->history[i] = hist[i];
      for (int i = m; i < info->history_cap; ++i) info->history[i] = 0.0;
    }
  }
  if (fallback_it >= 0) TRY(capture_vcycle_graphs(h, s));
  return 0;
}

int sgmg_fgmres_solve(sgmg_hierarchy* h, int precond, int restart, const double* f, double* u,
                      double rtol, int maxit, sgmg_solve_info* info, void* stream) {
  if (!h || !f || !u) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (precond < 0 || precond > 2 || maxit < 0) { set_error("bad precond or maxit"); return SGMG_EINVAL; }
  if (restart < 1 || restart >= basis_max_cols()) {
    set_error("restart must be in 1.." + std::to_string(basis_max_cols() - 1));
    return SGMG_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  const Level& L0 = h->lev[0];
  const int n = L0.g.n;
  const int m = restart;
  if (h->kry_cols < m) {
    if (h->kry) hipFree(h->kry);
    h->kry = nullptr;
    h->kry_cols = 0;
    if (hipMalloc(&h->kry, (size_t)(2 * m + 1) * n * sizeof(double)) != hipSuccess) {
      h->kry = nullptr;
      set_error("FGMRES basis allocation failed");
      return SGMG_ENOMEM;
    }
    h->kry_cols = m;
  }
  if (!h->kry_small && hipMalloc(&h->kry_small, 4 * 64 * sizeof(double)) != hipSuccess) {
    h->kry_small = nullptr;
    set_error("FGMRES allocation failed");
    return SGMG_ENOMEM;
  }
  double* V = h->kry;                                  // columns 0..m
  double* Z = h->kry + (size_t)(m + 1) * n;            // columns 0..m-1
  double* h1 = h->kry_small;                            // first Gram-Schmidt pass
  double* h2 = h->kry_small + 64;                       // second pass
  double* hw = h->kry_small + 128;                      // ||w||^2 ; ||r||^2 at cycle starts
  double* yd = h->kry_small + 192;
  double hbuf[193];
  hipEvent_t e0, e1;
  SGMG_HIP(hipEventCreate(&e0));
  SGMG_HIP(hipEventCreate(&e1));
  SGMG_HIP(hipEventRecord(e0, s));
  auto K64 = [&](const double* x, double* y) {
    return apply_level<double>(h, 0, SGMG_F64, x, epi_store<double>(y), s);
  };
  auto precondition = [&](const double* r, double* z) -> int {
    if (precond == 2) return vcycle_full(h, r, z, s);
    if (precond == 1) launch_apply_dinv(L0.dinv64, r, z, n, s);
    else launch_copy(r, z, n, s);
    return check_launch();
  };
  auto read = [&](const double* src, int count, double* dst) -> int {
    SGMG_HIP(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipStreamSynchronize(s));
    return 0;
  };
  int rc = 0, status = SGMG_MAXIT, it = 0;
  double nf = 0.0, rel = 0.0, rel_true = -1.0;
  std::vector<double> hist;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  auto Hat = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  launch_copy(u, h->xs, n, s);
  launch_dot(f, f, nullptr, n, h->ws, hw, s);
  if ((rc = check_launch()) || (rc = read(hw, 1, hbuf))) goto done;
  nf = std::sqrt(hbuf[0]);
  if (nf == 0.0) {
    SGMG_HIP(hipMemsetAsync(h->xs, 0, (size_t)n * sizeof(double), s));
    status = SGMG_CONVERGED; rel = rel_true = 0.0;
    hist.push_back(0.0);
    goto done;
  }
  for (;;) {
    // cycle start: true residual into V_0
    if ((rc = K64(h->xs, h->tmp))) break;
    launch_residual(f, h->tmp, V, n, h->ws, hw, s);
    if ((rc = check_launch()) || (rc = read(hw, 1, hbuf))) break;
    const double beta = std::sqrt(hbuf[0]);
    rel = rel_true = beta / nf;
    hist.push_back(rel);
    if (!std::isfinite(rel)) { status = SGMG_NONFINITE; break; }
    if (rel < rtol) { status = SGMG_CONVERGED; break; }
    if (it >= maxit) { status = SGMG_MAXIT; break; }
    launch_scale_inv_sqrt(V, V, hw, n, s);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool bad = false;
    for (int j = 0; j < m && it < maxit; ++j) {
      double* vj = V + (size_t)j * n;
      double* zj = Z + (size_t)j * n;
      double* w = V + (size_t)(j + 1) * n;
      if ((rc = precondition(vj, zj))) break;
      if ((rc = K64(zj, w))) break;
      // classical Gram-Schmidt with one reorthogonalisation (two passes)
      launch_basis_dots(V, j + 1, w, n, h->ws, h1, s);
      launch_basis_update(w, V, j + 1, h1, n, 1, h->ws, h2, s);
      launch_basis_update(w, V, j + 1, h2, n, 0, h->ws, hw, s);
      if ((rc = check_launch()) || (rc = read(h->kry_small, 129, hbuf))) break;
      for (int i = 0; i <= j; ++i) Hat(i, j) = hbuf[i] + hbuf[64 + i];
      const double hnext = std::sqrt(hbuf[128]);
      Hat(j + 1, j) = hnext;
      ++it;
      k = j + 1;
      for (int i = 0; i < j; ++i) {                    // earlier rotations on column j
        const double a = Hat(i, j), b = Hat(i + 1, j);
        Hat(i, j) = cs[i] * a + sn[i] * b;
        Hat(i + 1, j) = -sn[i] * a + cs[i] * b;
      }
      const double a = Hat(j, j), b = Hat(j + 1, j);
      const double d = std::hypot(a, b);
      cs[j] = d > 0.0 ? a / d : 1.0;
      sn[j] = d > 0.0 ? b / d : 0.0;
      Hat(j, j) = d;
      Hat(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      rel = std::fabs(g[j + 1]) / nf;
      hist.push_back(rel);
      if (!std::isfinite(rel)) { bad = true; break; }
      if (hnext < 1e-14 || rel < rtol) break;
      launch_scale_inv_sqrt(w, w, hw, n, s);
    }
    if (rc) break;
    if (bad) { status = SGMG_NONFINITE; break; }
    if (k == 0) break;
    // R y = g (back substitution; least squares on a singular diagonal)
    bool singular = false;
    for (int i = 0; i < k; ++i) singular = singular || Hat(i, i) == 0.0;
    if (!singular) {
      for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int c = i + 1; c < k; ++c) t -= Hat(i, c) * y[c];
        y[i] = t / Hat(i, i);
      }
    } else {
      // rank-deficient R (an exactly vanishing rotated diagonal): a basic
      // least-squares solution, the columns with R_ii = 0 left out
      for (int i = k - 1; i >= 0; --i) {
        if (Hat(i, i) == 0.0) { y[i] = 0.0; continue; }
        double t = g[i];
        for (int c = i + 1; c < k; ++c) t -= Hat(i, c) * y[c];
        y[i] = t / Hat(i, i);
      }
    }
    SGMG_HIP(hipMemcpyAsync(yd, y.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
    launch_basis_combine(h->xs, Z, k, yd, n, s);
    if ((rc = check_launch())) break;
  }
done:
  if (rc) {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
  }
  launch_copy(h->xs, u, n, s);
  SGMG_HIP(hipEventRecord(e1, s));
  SGMG_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (info) {
    info->status = status;
    info->iters = it;
    info->rel_res_true = rel_true;
    info->rel_res_recur = rel;
    info->solve_ms = ms;
    info->fallback_iter = -1;
    if (info->history && info->history_cap > 0) {
      const int mm = std::min<int>(info->history_cap, (int)hist.size());
      for (int i = 0; i < mm; ++i) info->history[i] = hist[i];
      for (int i = mm; i < info->history_cap; ++i) info->history[i] = 0.0;
    }
  }
  return 0;
}

int sgmg_set_launch_shape(sgmg_hierarchy* h, int variant, int rows, int planes) {
  if (!h) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (variant == 3) {
    // level 1: rows 0 the stored stencil, rows 1 the element products
    if (!h->l1_E8 || rows < 0 || rows > 1 || (rows == 1 && planes < 1)) {
      set_error("level-1 shape must be (0, any) or (1, planes >= 1) on a hierarchy with the "
                "level-1 element products (FP64 level 1 above the coarsest, stencil_form 0 or 3)");
      return SGMG_EINVAL;
    }
    h->l1_mf = rows == 1;
    if (rows == 1) h->l1_zchunk = planes;
    for (auto& row : h->iter_graph)
      for (auto& g : row)
        if (g) { hipGraphExecDestroy(g); g = nullptr; }
    return 0;
  }
  if (variant < 0 || variant > 2) { set_error("variant must be 0 (BF16), 1 (BF16X3), 2 (FP64) or 3 (level 1)"); return SGMG_EINVAL; }
  const bool node64 = variant == 2 && rows == 0 && planes == 0;
  const bool sf64 = variant == 2 && rows == 1 && planes >= 1;
  if (!node64 && !sf64 && !mfma_shape_valid(rows, planes)) {
    set_error("shape must have rows 4 or 8 and planes >= 1 (FP64 also (0, 0) and (1, planes >= 1))");
    return SGMG_EINVAL;
  }
  h->mfma_rows[variant] = rows;
  h->mfma_zchunk[variant] = planes;
  for (auto& row : h->iter_graph)        // captured graphs hold the old launch shape
    for (auto& g : row)
      if (g) { hipGraphExecDestroy(g); g = nullptr; }
  return 0;
}

namespace {

// Number of eigenvalues of the symmetric tridiagonal T (diagonal d, off-
// diagonal e) below x: the sign changes of its LDL^T pivots (Sturm count).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int c = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    q = d[i] - x - (i ? e[i - 1] * e[i - 1] / q : 0.0);
    if (q == 0.0) q = -1e-300;            // x on a pivot: count it below
    if (q < 0.0) ++c;
  }
  return c;
}

// k-th smallest eigenvalue (k = 1..n) by bisection inside the Gershgorin bounds.
double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int k) {
  double lo = d[0], hi = d[0];
  for (size_t i = 0; i < d.size(); ++i) {
    const double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < d.size() ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  for (int it = 0; it < 400; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(d, e, mid) >= k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

int sgmg_lanczos(sgmg_hierarchy* h, int precond, int m, const double* g, double breakdown,
                 double* alpha, double* beta, int* steps, double* ritz, void* stream) {
  if (!h || !g || !alpha || !beta || !steps) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (m < 1 || precond < 0 || precond > 2 || !(breakdown >= 0.0)) {
    set_error("bad Lanczos arguments");
    return SGMG_EINVAL;
  }
  *steps = 0;
  hipStream_t s = as_stream(stream);
  const Level& L0 = h->lev[0];
  const int n = L0.g.n;
  double* r = h->r;
  double* z = h->z;
  double* v = h->p;
  double* w = h->r_old;
  double* wp = h->tmp;
  double* sv = h->q;
  auto precondition = [&](const double* x, double* y) -> int {
    if (precond == 2) return vcycle_full(h, x, y, s);
    if (precond == 1) launch_apply_dinv(L0.dinv64, x, y, n, s);
    else launch_copy(x, y, n, s);
    return check_launch();
  };
  auto dot = [&](const double* a, const double* b, double* out) -> int {
    launch_dot(a, b, nullptr, n, h->ws, h->sc + SC_XW, s);
    TRY(check_launch());
    SGMG_HIP(hipMemcpyAsync(h->h_sc, h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipStreamSynchronize(s));
    *out = h->h_sc[SC_XW];
    return 0;
  };
  launch_lanczos_start(g, L0.fixn, r, n, s);
  TRY(precondition(r, z));
  double rz = 0.0;
  TRY(dot(r, z, &rz));
  if (!(rz > 0.0) || !std::isfinite(rz)) {
    set_error("start vector has r.Mr <= 0 or is not finite");
    return SGMG_EINVAL;
  }
  const double b1 = std::sqrt(rz);
  launch_lanczos_next(r, z, b1, w, v, n, s);
  SGMG_HIP(hipMemsetAsync(wp, 0, (size_t)n * sizeof(double), s));
  double b = 0.0, amax = 0.0;
  int k = 0;
  for (; k < m;) {
    TRY(apply_level<double>(h, 0, SGMG_F64, v, epi_store<double>(sv), s));
    double a = 0.0;
    TRY(dot(sv, v, &a));
    launch_lanczos_resid(sv, w, wp, a, b, r, n, s);
    TRY(precondition(r, z));
    TRY(dot(r, z, &rz));
    const double bn = rz > 0.0 ? std::sqrt(rz) : 0.0;
    alpha[k] = a;
    beta[k] = bn;
    amax = std::max(amax, std::fabs(a));
    ++k;
    if (!std::isfinite(a) || !std::isfinite(bn)) {
      *steps = k;
      set_error("Lanczos produced a non-finite coefficient");
      return SGMG_EINVAL;
    }
    if (!(bn > breakdown * amax)) break;
    std::swap(w, wp);                      // w_prev <- w; w and v are rewritten below
    launch_lanczos_next(r, z, bn, w, v, n, s);
    b = bn;
  }
  *steps = k;
  if (ritz) {
    std::vector<double> d(alpha, alpha + k), e(beta, beta + (k > 0 ? k - 1 : 0));
    ritz[0] = tridiag_eig(d, e, 1);
    ritz[1] = tridiag_eig(d, e, k);
  }
  SGMG_HIP(hipStreamSynchronize(s));
  return 0;
}

int sgmg_autotune(sgmg_hierarchy* h, int* shape_out, void* stream) {
  if (!h) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (!h->kt.integral) { set_error("MFMA path unavailable for this nu"); return SGMG_EINVAL; }
  hipStream_t s = as_stream(stream);
  const Level& L0 = h->lev[0];
  float *u = nullptr, *y = nullptr;
  SGMG_HIP(hipMalloc(&u, (size_t)L0.g.n * sizeof(float)));
  if (hipMalloc(&y, (size_t)L0.g.n * sizeof(float)) != hipSuccess) {
    hipFree(u);
    set_error("autotune allocation failed");
    return SGMG_ENOMEM;
  }
  hipMemsetAsync(u, 0, (size_t)L0.g.n * sizeof(float), s);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  const int rows_c[] = {4, 8};
  const int z_c[] = {2, 3, 4, 6, 8, 16, 32};
  double* u64 = nullptr;
  double* y64 = nullptr;
  int rc = 0;
  if (hipMalloc(&u64, (size_t)L0.g.n * sizeof(double)) != hipSuccess ||
      hipMalloc(&y64, (size_t)L0.g.n * sizeof(double)) != hipSuccess) {
    set_error("autotune allocation failed");
    rc = SGMG_ENOMEM;
  } else {
    hipMemsetAsync(u64, 0, (size_t)L0.g.n * sizeof(double), s);
    hipMemsetAsync(y64, 0, (size_t)L0.g.n * sizeof(double), s);
  }
  // variant q: 0 BF16, 1 BF16X3, 2 FP64
  for (int q = 0; q < 3 && !rc; ++q) {
    if (q == 2 && !mfma64_size_ok(L0.g)) break;
    const int key = q == 2 ? 64 : (q ? 3 : 1);
    int best_r = 8, best_z = 8;
    float best_ms = 1e30f;
    if (q == 2) {                                 // vector-ALU node kernel (rows 0)
      for (int w = 0; w < 3; ++w)
        launch_apply_fine_node<double>(L0.g, h->E64, h->ke64, u64, L0.fixn, epi_store<double>(y64), s);
      hipEventRecord(e0, s);
      for (int r = 0; r < 20; ++r)
        launch_apply_fine_node<double>(L0.g, h->E64, h->ke64, u64, L0.fixn, epi_store<double>(y64), s);
      hipEventRecord(e1, s);
      if ((rc = check_launch())) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = SGMG_EHIP;
        set_error("autotune sync failed");
        break;
      }
      hipEventElapsedTime(&best_ms, e0, e1);
      best_r = best_z = 0;
      // vector-ALU sum-factorised tiles (rows 1)
      for (int z : z_c) {
        if (z > L0.g.Nz && z != z_c[0]) continue;
        for (int w = 0; w < 3; ++w)
          launch_apply_fine_sf64(L0.g, z, h->E64, h->kt.lam, h->kt.mu, u64, L0.fixn,
                                 epi_store<double>(y64), s);
        hipEventRecord(e0, s);
        for (int r = 0; r < 20; ++r)
          launch_apply_fine_sf64(L0.g, z, h->E64, h->kt.lam, h->kt.mu, u64, L0.fixn,
                                 epi_store<double>(y64), s);
        hipEventRecord(e1, s);
        if ((rc = check_launch())) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = SGMG_EHIP;
          set_error("autotune sync failed");
          break;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) { best_ms = ms; best_r = 1; best_z = z; }
      }
      if (rc) break;
    }
    for (int rows : rows_c) {
      for (int z : z_c) {
        if (z > L0.g.Nz && z != z_c[0]) continue;
        auto launch = [&]() {
          if (q == 2)
            launch_apply_fine_mfma64(L0.g, rows, z, h->E64, h->atab64, u64, L0.fixn,
                                     epi_store<double>(y64), s);
          else   // a Chebyshev smoothing step: the epilogue of most V-cycle applications
            launch_apply_fine_mfma(L0.g, key, rows, z, h->E32s, h->atab, u, L0.fixn,
                                   epi_smooth<float>(y, u, (const float*)u64, (float*)y64, 0.5,
                                                     0.5, 1, nullptr),
                                   s);
        };
        for (int w = 0; w < 3; ++w) launch();
        hipEventRecord(e0, s);
        for (int r = 0; r < 30; ++r) launch();
        hipEventRecord(e1, s);
        if ((rc = check_launch())) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = SGMG_EHIP;
          set_error("autotune sync failed");
          break;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) { best_ms = ms; best_r = rows; best_z = z; }
      }
      if (rc) break;
    }
    if (rc) break;
    h->mfma_rows[q] = best_r;
    h->mfma_zchunk[q] = best_z;
    if (shape_out) { shape_out[2 * q] = best_r; shape_out[2 * q + 1] = best_z; }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(L0.g.nx, L0.g.ny, L0.g.nz, key)] = std::make_pair(best_r, best_z);
  }
  // level 1: the stored stencil against the element products (1 to 6 and
  // 8 planes); with stencil_form 3 the products stay and only their chunk
  // length is chosen
  if (!rc && h->l1_E8) {
    const Level& L1 = h->lev[1];
    const bool keep_mf = h->o.stencil_form == 3;
    float best_ms = 1e30f;
    int best = 0, best_z = h->l1_zchunk;
    const int zl[] = {0, 1, 2, 3, 4, 5, 6, 8};   // 0: the stencil
    for (int z : zl) {
      if (z == 0 && keep_mf) continue;
      if (z > L1.g.Nz && z != 2) continue;
      h->l1_mf = z > 0;
      if (z > 0) h->l1_zchunk = z;
      for (int w = 0; w < 3 && !rc; ++w)
        rc = apply_level<double>(h, 1, SGMG_F64, u64, epi_store<double>(y64), s);
      hipEventRecord(e0, s);
      for (int r = 0; r < 20 && !rc; ++r)
        rc = apply_level<double>(h, 1, SGMG_F64, u64, epi_store<double>(y64), s);
      hipEventRecord(e1, s);
      if (rc) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = SGMG_EHIP;
        set_error("autotune sync failed");
        break;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (ms < best_ms) { best_ms = ms; best = z > 0; best_z = z > 0 ? z : best_z; }
    }
    h->l1_mf = best == 1;
    h->l1_zchunk = best_z;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(L0.g.nx, L0.g.ny, L0.g.nz, 101)] = std::make_pair(best, best_z);
  }
  hipStreamSynchronize(s);
  if (u64) hipFree(u64);
  if (y64) hipFree(y64);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamSynchronize(s);
  hipFree(u);
  hipFree(y);
  // captured iteration graphs hold the old launch shape: capture them again
  // here, so that no later solve has to capture
  for (auto& row : h->iter_graph)
    for (auto& g : row)
      if (g) { hipGraphExecDestroy(g); g = nullptr; }
  if (!rc) rc = capture_vcycle_graphs(h, s);
  return rc;
}

int sgmg_num_levels(const sgmg_hierarchy* h) { return h ? h->L : 0; }

int sgmg_unet_input(const sgmg_hierarchy* h, const double* rho, const double* f, int Dp, int Hp,
                    int Wp, float* in, void* stream) {
  if (!h || !rho || !f || !in) { set_error("NULL argument"); return SGMG_EINVAL; }
  const Grid& g = h->lev[0].g;
  if (Dp < g.Nz || Hp < g.Ny || Wp < g.Nx) { set_error("padded volume smaller than the node grid"); return SGMG_EINVAL; }
  launch_unet_input(g, rho, f, h->lev[0].fixn, h->sc + SC_MAX, Dp, Hp, Wp, in, as_stream(stream));
  return check_launch();
}

int sgmg_unet_output(const sgmg_hierarchy* h, const float* out, int Dp, int Hp, int Wp, double* u0,
                     void* stream) {
  if (!h || !out || !u0) { set_error("NULL argument"); return SGMG_EINVAL; }
  const Grid& g = h->lev[0].g;
  if (Dp < g.Nz || Hp < g.Ny || Wp < g.Nx) { set_error("padded volume smaller than the node grid"); return SGMG_EINVAL; }
  launch_unet_output(g, out, h->lev[0].fixn, Dp, Hp, Wp, u0, as_stream(stream));
  return check_launch();
}

int sgmg_unet_target(const sgmg_hierarchy* h, const double* u, int Dp, int Hp, int Wp, float* t,
                     float* mask, void* stream) {
  if (!h || !u || !t) { set_error("NULL argument"); return SGMG_EINVAL; }
  const Grid& g = h->lev[0].g;
  if (Dp < g.Nz || Hp < g.Ny || Wp < g.Nx) { set_error("padded volume smaller than the node grid"); return SGMG_EINVAL; }
  launch_unet_target(g, u, h->sc + SC_MAX, Dp, Hp, Wp, t, mask, as_stream(stream));
  return check_launch();
}

int sgmg_warm_start_scale(sgmg_hierarchy* h, const double* f, double* u0, double* alpha,
                          void* stream) {
  if (!h || !f || !u0) { set_error("NULL argument"); return SGMG_EINVAL; }
  hipStream_t s = as_stream(stream);
  const int n = h->lev[0].g.n;
  launch_dot(f, u0, nullptr, n, h->ws, h->sc + SC_XW, s);
  TRY(apply_level<double>(h, 0, SGMG_F64, u0, epi_store<double>(h->tmp, h->ws, h->sc + SC_XDX), s));
  launch_scale_by_ratio(u0, n, h->sc + SC_XW, h->sc + SC_XDX, h->sc + SC_NRM, s);
  TRY(check_launch());
  if (alpha) {
    SGMG_HIP(hipMemcpyAsync(alpha, h->sc + SC_NRM, sizeof(double), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipStreamSynchronize(s));
  }
  return 0;
}

}  // extern "C"

// ===========================================================================
// Allocation-free warm-start scaling.  The reduction partials and the three
// scalars of sgmg_warm_start_scale live in this fixed device array instead of
// the hierarchy's workspace, and the product K u0 is reduced without being
// stored, so the call allocates nothing and never synchronises.  Every GPU the
// library runs on holds its own copy until the process ends; every slot a call
// reads is written earlier in the same call (nothing needs clearing), and
// calls that overlap on one GPU race on it.
static constexpr size_t kScratchPartials = size_t(1) << 16;   // block partials (doubles)
static constexpr size_t kScratchScalars = 32;                 // num, den, alpha, padding
static __device__ __align__(256) double scratch[kScratchPartials + kScratchScalars];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kScratchDevices] = {};

// Device address of the current device's copy of the array.  The array's
// name is a host-side stand-in in host code: only this address may be passed
// to kernels or copies.
int scratch_address(double** out) {
  int dev = -1;
  SGMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) {
    set_error("device index out of range for the static scratch table");
    return SGMG_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return SGMG_EHIP;
    }
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return 0;
}

}  // namespace

extern "C" {

int sgmg_warm_start_scale_noalloc(const sgmg_hierarchy* h, const double* f, double* u0,
                                  double* alpha_dev, void* stream) {
  if (!h || !f || !u0) { set_error("NULL argument"); return SGMG_EINVAL; }
  const int n = h->lev[0].g.n;
  const size_t need = std::max<size_t>((size_t)k64_dot_partials(h), (size_t)vec_dot_blocks(n));
  if (need > kScratchPartials) {
    set_error("mesh too large for the static scratch: " + std::to_string(need) +
              " reduction partials needed, at most " + std::to_string(kScratchPartials));
    return SGMG_EINVAL;
  }
  double* ptr = nullptr;
  TRY(scratch_address(&ptr));
  hipStream_t s = as_stream(stream);
  const RedWs ws{ptr, nullptr};
  double* num = ptr + kScratchPartials;
  double* den = num + 1;
  double* alpha = num + 2;
  launch_dot(f, u0, nullptr, n, ws, num, s);
  // u0 . K u0 from the FP64 operator's block partials; its output is not stored
  TRY(apply_level<double>(h, 0, SGMG_F64, u0, epi_store<double>(nullptr, ws, den), s));
  launch_scale_by_ratio(u0, n, num, den, alpha_dev ? alpha_dev : alpha, s);
  return check_launch();
}

}  // extern "C"

// ===========================================================================
// Batched persistent solver (BASELINE extension: many systems, one launch)
struct sgmg_batch {
  std::vector<sgmg_hierarchy*> hs;
  BSys* d_sys = nullptr;
  // work vectors of the cached item set
  std::vector<int> items_sys;
  std::vector<void*> item_mem;
  std::vector<BItem> h_items;     // in execution (largest-first) order
  std::vector<int> order;         // execution slot -> caller item index
  BItem* d_items = nullptr;
  int* d_queue = nullptr;
  BOut* d_out = nullptr;
  BOut* h_out = nullptr;
  int bs = 0;                     // tuned block size (0: not tuned yet)
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  int g_nitems = -1, g_maxit = -1, g_bs = -1;
  double g_rtol = -1.0;
  // stage-batched solve of the cached item set: stage tables, per-item
  // partials, scalars and active flags, the prologue and iteration graphs
  struct Staged {
    bool ready = false;
    void* dmem = nullptr;
    BsTable tv, ts[8], tr[8], tcg, tcm;
    BsTable tsc[8];                // levels >= 1: row-split stencil blocks
    BsTable tss[8];                // levels >= 1: LDS-staged stencil blocks
    int lform[8] = {};             // per level: 1 = LDS-staged form (timed faster)
    double* part = nullptr;
    double* scal = nullptr;
    int* flags = nullptr;          // [0, n): prologue, [n, 2n): iteration
    int* h_flags = nullptr;        // pinned mirror
    double* h_scal = nullptr;      // pinned mirror
    int Lmax = 0, steps0 = 0, stepsL = 0;
    hipGraphExec_t g_pro = nullptr, g_it = nullptr;
    // level 0 on the BF16X3 MFMA operator: launch shape, (item, block)
    // table and per-item tile grids
    bool mfma0 = false;
    int mrows = 0, mz = 0;
    BsTable tm0;
    const int4* geo = nullptr;
    void* mdmem = nullptr;
    // the outer FP64 K p on the FP64 MFMA operator: launch shape, table
    // (with per-item start / count for the p.q finalize) and tile grids
    bool mfma64 = false;
    int k64rows = 0, k64z = 0;
    BsTable tk64;
    const int4* geo64 = nullptr;
    void* m64dmem = nullptr;
    // one-launch solve: device-side iteration control (arrays in lmem, a
    // pinned mirror) and the loop graphs: g_first = prologue + decision +
    // l_steps iterations, g_more = l_steps further iterations
    BsLoop lp{};
    void* lmem = nullptr;
    void* h_lmem = nullptr;
    size_t lbytes = 0;
    hipGraphExec_t g_first = nullptr, g_more = nullptr;
    int l_steps = 0, l_maxit = -1;
    double l_rtol = -1.0;
  } st;
};

namespace {

void batch_drop_graph(sgmg_batch* b) {
  if (b->graph) hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
}

void batch_free_staged(sgmg_batch* b) {
  auto& st = b->st;
  if (st.g_pro) hipGraphExecDestroy(st.g_pro);
  if (st.g_it) hipGraphExecDestroy(st.g_it);
  if (st.g_first) hipGraphExecDestroy(st.g_first);
  if (st.g_more) hipGraphExecDestroy(st.g_more);
  if (st.lmem) hipFree(st.lmem);
  if (st.h_lmem) hipHostFree(st.h_lmem);
  if (st.dmem) hipFree(st.dmem);
  if (st.mdmem) hipFree(st.mdmem);
  if (st.m64dmem) hipFree(st.m64dmem);
  if (st.h_flags) hipHostFree(st.h_flags);
  if (st.h_scal) hipHostFree(st.h_scal);
  st = sgmg_batch::Staged{};
}

void batch_free_items(sgmg_batch* b) {
  batch_free_staged(b);
  for (void* p : b->item_mem) hipFree(p);
  b->item_mem.clear();
  b->h_items.clear();
  b->items_sys.clear();
  if (b->d_items) hipFree(b->d_items);
  if (b->d_out) hipFree(b->d_out);
  if (b->h_out) hipHostFree(b->h_out);
  b->d_items = nullptr;
  b->d_out = nullptr;
  b->h_out = nullptr;
  batch_drop_graph(b);
}

BSys make_bsys(const sgmg_hierarchy* h) {
  BSys S{};
  S.L = h->L;
  for (int l = 0; l < h->L; ++l) {
    const Level& V = h->lev[l];
    BLevel& B = S.lev[l];
    B.g = V.g;
    B.fixn = V.fixn;
    B.dinv64 = V.dinv64;
    B.dinv32 = V.dinv32;
    B.S64 = V.S64;
    if (l < h->L - 1) {
      const Smoother sm = smoother_of(h, l);
      B.cheb = sm.cheb;
      B.steps = sm.steps;
      B.omega = sm.omega;
      B.theta = sm.theta;
      B.delta = sm.delta;
      B.sigma1 = sm.sigma1;
    }
  }
  S.E32 = h->E32;
  S.E32s = h->E32s;
  S.atab = h->atab;
  S.ke32 = h->ke32;
  S.E64 = h->E64;
  S.atab64 = h->atab64;
  S.lam = h->kt.lam;
  S.mu = h->kt.mu;
  S.ke64 = h->ke64;
  S.nL = h->nL;
  S.free_idx = h->free_idx;
  S.Ainv = h->Ainv;
  return S;
}

// Sub-buffers of one batch item's work memory (see sgmg_batch_item_layout).
constexpr int kMaxLevels = 8;
constexpr int kItemBufs = 10 + 4 * (kMaxLevels - 1) + 1;

// (Re)allocates the work vectors when the item set changes.
int batch_prepare_items(sgmg_batch* b, int nitems, const int* item_sys, hipStream_t s) {
  std::vector<int> key(item_sys, item_sys + nitems);
  if (key == b->items_sys && b->d_items) return 0;
  batch_free_items(b);
  b->items_sys = key;
  // largest systems first (longest-processing-time order for the queue)
  b->order.resize(nitems);
  for (int i = 0; i < nitems; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
    return b->hs[item_sys[a]]->lev[0].g.n > b->hs[item_sys[c]]->lev[0].g.n;
  });
  b->h_items.assign(nitems, BItem{});
  for (int k = 0; k < nitems; ++k) {
    const int sys = item_sys[b->order[k]];
    const sgmg_hierarchy* h = b->hs[sys];
    BItem& I = b->h_items[k];
    I.sys = sys;
    int ndofs[kMaxLevels];
    for (int l = 0; l < h->L; ++l) ndofs[l] = h->lev[l].g.n;
    size_t off[kItemBufs], sz[kItemBufs];
    const size_t bytes = sgmg_batch_item_layout(h->L, ndofs, h->nL, off, sz);
    if (!bytes) { set_error("batch item layout: bad level sizes"); return SGMG_EINVAL; }
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) { set_error("batch work allocation failed"); return SGMG_ENOMEM; }
    b->item_mem.push_back(mem);
    SGMG_HIP(hipMemsetAsync(mem, 0, bytes, s));
    char* c = (char*)mem;
    int k2 = 0;
    auto take = [&]() { return (void*)(c + off[k2++]); };
    I.r = (double*)take(); I.z = (double*)take(); I.p = (double*)take();
    I.q = (double*)take(); I.t = (double*)take();
    I.b0 = (float*)take(); I.d0 = (float*)take(); I.r0 = (float*)take();
    I.x0[0] = (float*)take(); I.x0[1] = (float*)take();
    for (int l = 1; l < h->L; ++l) {
      I.lb[l] = (double*)take();
      I.lx[l][0] = (double*)take();
      I.lx[l][1] = (double*)take();
      I.lr[l] = (double*)take();
    }
    I.rc = (double*)take();
  }
  SGMG_HIP(hipMalloc(&b->d_items, nitems * sizeof(BItem)));
  SGMG_HIP(hipMalloc(&b->d_out, nitems * sizeof(BOut)));
  SGMG_HIP(hipHostMalloc((void**)&b->h_out, nitems * sizeof(BOut), hipHostMallocDefault));
  SGMG_HIP(hipStreamSynchronize(s));
  return 0;
}

int batch_launch(sgmg_batch* b, int nitems, double rtol, int maxit, int bs, hipStream_t s) {
  const int grid = std::min(nitems, 1024);
  const bool same = b->graph && b->g_nitems == nitems && b->g_rtol == rtol &&
                    b->g_maxit == maxit && b->g_bs == bs;
  if (!same) {
    batch_drop_graph(b);
    if (!b->cap) SGMG_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    SGMG_HIP(hipStreamSynchronize(s));
    SGMG_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    launch_batch_pcg(bs, grid, b->d_sys, b->d_items, nitems, b->d_queue, b->d_out, rtol, maxit,
                     b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess) { set_error(std::string("batch capture: ") + hipGetErrorString(e)); return SGMG_EHIP; }
    const hipError_t e2 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) { b->graph = nullptr; set_error("batch graph instantiate failed"); return SGMG_EHIP; }
    b->g_nitems = nitems; b->g_rtol = rtol; b->g_maxit = maxit; b->g_bs = bs;
  }
  SGMG_HIP(hipGraphLaunch(b->graph, s));
  return 0;
}

// ---------------------------------------------------------------------------
// Stage-batched solve.
//   One V-cycle of every flagged item as a sequence of stage launches.  cur
//   bit l = ping-pong buffer of level l's iterate; every item has the same
//   smoothing step counts, so the sequence is the same for all of them; at
//   each level only items for which the level is above their coarsest take
//   part (tables ts, tr).
void bs_vcycle(const sgmg_batch::Staged& st, const BsArgs& a, const int* flags, hipStream_t s) {
  unsigned cur = 0u;
  auto cb = [&](int l) { return (int)((cur >> l) & 1u); };
  auto flip = [&](int l) { cur ^= 1u << l; };
  // Galerkin level l: the stencil form timed faster on the item set
  auto stencil = [&](int l, int mode, int cin) {
    if (st.lform[l]) bs_stencil_s(a, st.tss[l], flags, l, mode, cin, s);
    else bs_stencil(a, st.tsc[l], flags, l, mode, cin, s);
  };
  // level-0 smoothing step and residual: MFMA or vector-ALU operator
  auto smooth0 = [&](int post, int k, int cin, int last) {
    if (st.mfma0)
      bs_fine_mfma(a, st.tm0, st.geo, flags, st.mrows, st.mz, EPI_SMOOTH, post, k, cin, last, s);
    else
      bs_smooth0(a, st.ts[0], flags, post, k, cin, last, s);
  };
  for (int l = 0; l < st.Lmax - 1; ++l) {
    const int steps = l == 0 ? st.steps0 : st.stepsL;
    for (int k = 1; k < steps; ++k) {
      if (l == 0) smooth0(0, k, cb(0), 0);
      else stencil(l, EPI_SMOOTH, cb(l));
      flip(l);
    }
    if (l == 0 && st.mfma0) bs_fine_mfma(a, st.tm0, st.geo, flags, st.mrows, st.mz, EPI_RESID, 0, 0, cb(0), 0, s);
    else if (l == 0) bs_resid0(a, st.ts[0], flags, cb(0), s);
    else stencil(l, EPI_RESID, cb(l));
    bs_restrict(a, st.tr[l], flags, l, s);
    cur &= ~(1u << (l + 1));
  }
  bs_coarse(a, st.tcg, st.tcm, flags, s);
  for (int l = st.Lmax - 2; l >= 0; --l) {
    const int steps = l == 0 ? st.steps0 : st.stepsL;
    bs_prolong(a, st.ts[l], flags, l, cb(l), cb(l + 1), s);
    for (int k = 0; k < steps; ++k) {
      if (l == 0) smooth0(1, k, cb(0), k == steps - 1);
      else stencil(l, EPI_SMOOTH, cb(l));
      flip(l);
    }
  }
}

// Prologue (flags [0, n)): r = f - K u and (f.f, r.r), then z = V(r), p = z,
// rz.  It is also the true-residual check and restart of the iteration.
void bs_prologue(const sgmg_batch* b, const BsArgs& a, int n, hipStream_t s) {
  const auto& st = b->st;
  const int* fl = st.flags;
  bs_fine64_res(a, st.ts[0], fl, st.part, s);
  bs_finalize(st.ts[0], n, 2, st.part, fl, 0, st.scal, s);
  bs_entry(a, st.tv, fl, s);
  bs_vcycle(st, a, fl, s);
  bs_dot_rz(a, st.tv, fl, 1, st.part, s);
  bs_finalize(st.tv, n, 1, st.part, fl, 4, st.scal, s);
}

// One PCG iteration (flags [n, 2n)): q = K p, alpha, x and r, V-cycle, beta, p.
void bs_iteration(const sgmg_batch* b, const BsArgs& a, int n, hipStream_t s) {
  const auto& st = b->st;
  const int* fl = st.flags + n;
  if (st.mfma64) {
    bs_fine_mfma64_store_dot(a, st.tk64, st.geo64, fl, st.k64rows, st.k64z, st.part, s);
    bs_finalize(st.tk64, n, 1, st.part, fl, 1, st.scal, s);
  } else {
    bs_fine64_store_dot(a, st.ts[0], fl, st.part, s);
    bs_finalize(st.ts[0], n, 1, st.part, fl, 1, st.scal, s);
  }
  bs_update_xr(a, st.tv, fl, st.scal, st.part, s);
  bs_finalize(st.tv, n, 1, st.part, fl, 2, st.scal, s);
  bs_vcycle(st, a, fl, s);
  bs_dot_rz(a, st.tv, fl, 0, st.part, s);
  bs_finalize(st.tv, n, 1, st.part, fl, 3, st.scal, s);
  bs_update_p(a, st.tv, fl, st.scal, s);
}

template <class F>
int bs_capture_fn(sgmg_batch* b, F&& body, hipGraphExec_t* out) {
  if (!b->cap) SGMG_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  SGMG_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  body(BsArgs{b->d_sys, b->d_items}, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess) { set_error(std::string("staged batch capture: ") + hipGetErrorString(e)); return SGMG_EHIP; }
  const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e2 != hipSuccess) { *out = nullptr; set_error("staged batch graph instantiate failed"); return SGMG_EHIP; }
  return 0;
}

int bs_capture(sgmg_batch* b, void (*body)(const sgmg_batch*, const BsArgs&, int, hipStream_t),
               int n, hipGraphExec_t* out) {
  return bs_capture_fn(b, [&](const BsArgs& a, hipStream_t s) { body(b, a, n, s); }, out);
}

// steps PCG iterations under device-side control: after each iteration the
// decision kernel flags the items whose recurrence residual passed, the
// prologue (the true-residual check and restart) runs for them, and the
// second decision sets the next iteration's flags; items that stopped have
// no flag and their blocks return at once.  The launch ends with the true
// residual of the items that stopped without one, once no item iterates.
void bs_loop_steps(const sgmg_batch* b, const BsArgs& a, int n, int steps, double rtol, int maxit,
                   hipStream_t s) {
  const auto& st = b->st;
  for (int k = 0; k < steps; ++k) {
    bs_iteration(b, a, n, s);
    bs_decide_iter(n, st.scal, st.flags, st.lp, k & 1, rtol, maxit, s);
    bs_prologue(b, a, n, s);
    bs_decide_check(n, st.scal, st.flags, st.lp, k & 1, rtol, maxit, s);
  }
  bs_decide_final(n, st.flags, st.lp, s);
  bs_prologue(b, a, n, s);
  bs_final_rel(n, st.scal, st.flags, st.lp, s);
}

// The loop state and the two loop graphs of the one-launch solve (kept while
// the item set, rtol, maxit and steps stay the same).
int bs_prepare_loop(sgmg_batch* b, int n, double rtol, int maxit, int steps, hipStream_t s) {
  auto& st = b->st;
  if (!st.lmem) {
    const size_t ib = ((3 * (size_t)n + 2) * sizeof(int) + 255) & ~(size_t)255;
    st.lbytes = ib + 3 * (size_t)n * sizeof(double);
    if (hipMalloc(&st.lmem, st.lbytes) != hipSuccess ||
        hipHostMalloc(&st.h_lmem, st.lbytes, hipHostMallocDefault) != hipSuccess) {
      set_error("batch loop allocation failed");
      return SGMG_ENOMEM;
    }
    int* ip = (int*)st.lmem;
    double* dp = (double*)((char*)st.lmem + ib);
    st.lp = BsLoop{ip, ip + n, dp, dp + n, dp + 2 * n, ip + 2 * n, ip + 3 * n};
  }
  if (st.g_first && st.l_steps == steps && st.l_maxit == maxit && st.l_rtol == rtol) return 0;
  if (st.g_first) hipGraphExecDestroy(st.g_first);
  if (st.g_more) hipGraphExecDestroy(st.g_more);
  st.g_first = st.g_more = nullptr;
  SGMG_HIP(hipStreamSynchronize(s));
  TRY(bs_capture_fn(b, [&](const BsArgs& a, hipStream_t cs) {
    bs_loop_init(n, st.flags, st.lp, cs);
    bs_prologue(b, a, n, cs);
    bs_decide_start(n, st.scal, st.flags, st.lp, rtol, maxit, cs);
    bs_zero_u(a, st.tv, st.lp, cs);
    bs_loop_steps(b, a, n, steps, rtol, maxit, cs);
  }, &st.g_first));
  TRY(bs_capture_fn(b, [&](const BsArgs& a, hipStream_t cs) {
    bs_loop_steps(b, a, n, steps, rtol, maxit, cs);
  }, &st.g_more));
  st.l_steps = steps;
  st.l_maxit = maxit;
  st.l_rtol = rtol;
  return 0;
}

// Level 0 of the staged solve on the BF16X3 MFMA operator: for each
// candidate launch shape the (item, block) table and tile grids are built
// and the smoothing stage over all items is timed (HIP events, three
// launches after one warm-up, into the items' scratch vectors); the fastest
// shape's table stays.  st.flags[0, n) must be allocated.
int bs_tune_mfma(sgmg_batch* b, int n, hipStream_t s) {
  auto& st = b->st;
  constexpr int kShapes = 6;
  const int shapes[kShapes][2] = {{4, 2}, {4, 3}, {4, 4}, {8, 2}, {8, 3}, {8, 4}};
  std::vector<int2> tabs[kShapes];
  std::vector<int4> geos[kShapes];
  size_t maxe = 0;
  for (int c = 0; c < kShapes; ++c) {
    for (int i = 0; i < n; ++i) {
      const int4 gm = bs_mfma_geometry(b->hs[b->h_items[i].sys]->lev[0].g, shapes[c][0], shapes[c][1]);
      geos[c].push_back(gm);
      for (int j = 0; j < gm.w; ++j) tabs[c].push_back(int2{i, j});
    }
    maxe = std::max(maxe, tabs[c].size());
  }
  const size_t tb = (maxe * sizeof(int2) + 255) & ~(size_t)255;
  const size_t gb = ((size_t)n * sizeof(int4) + 255) & ~(size_t)255;
  char* m = nullptr;
  if (hipMalloc((void**)&m, tb + gb) != hipSuccess) {
    set_error("staged batch allocation failed");
    return SGMG_ENOMEM;
  }
  st.mdmem = m;
  int2* dtab = (int2*)m;
  int4* dgeo = (int4*)(m + tb);
  std::vector<int> ones(n, 1);
  SGMG_HIP(hipMemcpyAsync(st.flags, ones.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  SGMG_HIP(hipEventCreate(&e0));
  SGMG_HIP(hipEventCreate(&e1));
  const BsArgs a{b->d_sys, b->d_items};
  float best = 0.f;
  int bc = -1;
  for (int c = 0; c < kShapes; ++c) {
    SGMG_HIP(hipMemcpyAsync(dtab, tabs[c].data(), tabs[c].size() * sizeof(int2), hipMemcpyHostToDevice, s));
    SGMG_HIP(hipMemcpyAsync(dgeo, geos[c].data(), n * sizeof(int4), hipMemcpyHostToDevice, s));
    BsTable t;
    t.blk = dtab;
    t.n = (int)tabs[c].size();
    bs_fine_mfma(a, t, dgeo, st.flags, shapes[c][0], shapes[c][1], EPI_SMOOTH, 1, 1, 0, 0, s);
    SGMG_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r)
      bs_fine_mfma(a, t, dgeo, st.flags, shapes[c][0], shapes[c][1], EPI_SMOOTH, 1, 1, 0, 0, s);
    SGMG_HIP(hipEventRecord(e1, s));
    SGMG_HIP(hipEventSynchronize(e1));
    TRY(check_launch());
    float ms = 0.f;
    SGMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (bc < 0 || ms < best) { best = ms; bc = c; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  SGMG_HIP(hipMemcpyAsync(dtab, tabs[bc].data(), tabs[bc].size() * sizeof(int2), hipMemcpyHostToDevice, s));
  SGMG_HIP(hipMemcpyAsync(dgeo, geos[bc].data(), n * sizeof(int4), hipMemcpyHostToDevice, s));
  SGMG_HIP(hipStreamSynchronize(s));
  st.tm0 = BsTable{};
  st.tm0.blk = dtab;
  st.tm0.n = (int)tabs[bc].size();
  st.geo = dgeo;
  st.mrows = shapes[bc][0];
  st.mz = shapes[bc][1];
  return 0;
}

// Per Galerkin level, the smoothing stage over all items is timed in the
// row-split and the LDS-staged stencil forms (HIP events, three launches
// after one warm-up, into the items' scratch vectors) and the faster kept.
// st.flags[0, n) and the tables must be in place.
int bs_tune_stencil(sgmg_batch* b, int n, hipStream_t s) {
  auto& st = b->st;
  std::vector<int> ones(n, 1);
  SGMG_HIP(hipMemcpyAsync(st.flags, ones.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  SGMG_HIP(hipEventCreate(&e0));
  SGMG_HIP(hipEventCreate(&e1));
  const BsArgs a{b->d_sys, b->d_items};
  for (int l = 1; l < st.Lmax - 1; ++l) {
    float ms[2] = {0.f, 0.f};
    for (int form = 0; form < 2; ++form) {
      auto launch = [&]() {
        if (form) bs_stencil_s(a, st.tss[l], st.flags, l, EPI_SMOOTH, 0, s);
        else bs_stencil(a, st.tsc[l], st.flags, l, EPI_SMOOTH, 0, s);
      };
      launch();
      SGMG_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) launch();
      SGMG_HIP(hipEventRecord(e1, s));
      SGMG_HIP(hipEventSynchronize(e1));
      TRY(check_launch());
      SGMG_HIP(hipEventElapsedTime(&ms[form], e0, e1));
    }
    st.lform[l] = ms[1] < ms[0] ? 1 : 0;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return 0;
}

// Stage tables, partials, scalars and flags of the cached item set, and the
// two graphs.
int bs_prepare(sgmg_batch* b, int n, hipStream_t s) {
  auto& st = b->st;
  if (st.ready) return 0;
  const BSys* hs0 = nullptr;
  std::vector<BSys> hsys(b->hs.size());
  for (size_t k = 0; k < b->hs.size(); ++k) hsys[k] = make_bsys(b->hs[k]);
  st.Lmax = 0;
  for (int i = 0; i < n; ++i) {
    const BSys& S = hsys[b->h_items[i].sys];
    if (!hs0) hs0 = &S;
    if (S.lev[0].steps != hs0->lev[0].steps || (S.L > 2 && hs0->L > 2 && S.lev[1].steps != hs0->lev[1].steps)) {
      set_error("staged batch: all systems need the same smoothing step counts");
      return SGMG_EINVAL;
    }
    st.Lmax = std::max(st.Lmax, S.L);
  }
  st.steps0 = hs0->lev[0].steps;
  st.stepsL = 0;
  for (int i = 0; i < n; ++i) {
    const BSys& S = hsys[b->h_items[i].sys];
    if (S.L > 2) { st.stepsL = S.lev[1].steps; break; }
  }
  const int TB = bs_threads();
  // host tables: entries (item, local block), per-item start and count
  struct HT { std::vector<int2> blk; std::vector<int> start, count; };
  auto make = [&](auto nblocks) {
    HT t;
    t.start.resize(n);
    t.count.resize(n);
    for (int i = 0; i < n; ++i) {
      const int c = nblocks(hsys[b->h_items[i].sys]);
      t.start[i] = (int)t.blk.size();
      t.count[i] = c;
      for (int j = 0; j < c; ++j) t.blk.push_back(int2{i, j});
    }
    return t;
  };
  std::vector<HT> hts;
  hts.push_back(make([&](const BSys& S) { return div_up(S.lev[0].g.n, TB); }));        // tv
  for (int l = 0; l < st.Lmax - 1; ++l) {
    hts.push_back(make([&](const BSys& S) { return S.L - 1 > l ? div_up(S.lev[l].g.Nn, TB) : 0; }));
    hts.push_back(make([&](const BSys& S) { return S.L - 1 > l ? div_up(3 * S.lev[l + 1].g.Nn, TB) : 0; }));
  }
  hts.push_back(make([&](const BSys& S) { return div_up(S.nL, TB); }));               // tcg
  hts.push_back(make([&](const BSys& S) { return div_up(S.nL, bs_coarse_rows()); }));  // tcm
  for (int l = 1; l < st.Lmax - 1; ++l) {                                                // tsc, tss
    hts.push_back(make([&](const BSys& S) { return S.L - 1 > l ? bs_stencil_blocks(S.lev[l].g) : 0; }));
    hts.push_back(make([&](const BSys& S) { return S.L - 1 > l ? bs_stencil_s_blocks(S.lev[l].g) : 0; }));
  }
  // the outer K p on the FP64 MFMA operator when every item's fine level
  // fits it: one table per candidate launch shape (tuned below)
  // (rows 1: the vector-ALU sum/difference-basis operator, whose tiles are
  // those of rows 4)
  static constexpr int kK64 = 9;
  static const int k64_shapes[kK64][2] = {{4, 2}, {4, 4}, {4, 8}, {8, 4}, {1, 2}, {1, 3}, {1, 4},
                                          {1, 6}, {1, 8}};
  auto geo_rows = [](int r) { return r == 1 ? 4 : r; };
  bool mf64 = true;
  for (int i = 0; i < n; ++i) {
    const sgmg_hierarchy* h = b->hs[b->h_items[i].sys];
    mf64 = mf64 && h->atab64 && mfma64_size_ok(h->lev[0].g);
  }
  if (mf64)
    for (int c = 0; c < kK64; ++c)
      hts.push_back(make([&](const BSys& S) {
        return bs_mfma_geometry(S.lev[0].g, geo_rows(k64_shapes[c][0]), k64_shapes[c][1]).w;
      }));
  auto a16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
  size_t bytes = 0, maxblk = 0;
  for (const HT& t : hts) {
    bytes += a16(t.blk.size() * sizeof(int2)) + 2 * a16((size_t)n * sizeof(int));
    maxblk = std::max(maxblk, t.blk.size());
  }
  bytes = (bytes + 255) & ~(size_t)255;
  const size_t part_b = 2 * maxblk * sizeof(double);
  const size_t scal_b = (size_t)n * kBsScalars * sizeof(double);
  const size_t flag_b = 2 * (size_t)n * sizeof(int);
  char* m = nullptr;
  if (hipMalloc((void**)&m, bytes + part_b + scal_b + flag_b + 512) != hipSuccess) {
    set_error("staged batch allocation failed");
    return SGMG_ENOMEM;
  }
  st.dmem = m;
  size_t at = 0;
  std::vector<BsTable> dts;
  for (const HT& t : hts) {
    BsTable d;
    d.n = (int)t.blk.size();
    d.blk = (const int2*)(m + at);
    if (!t.blk.empty())
      SGMG_HIP(hipMemcpyAsync(m + at, t.blk.data(), t.blk.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    at += a16(t.blk.size() * sizeof(int2));
    d.start = (const int*)(m + at);
    SGMG_HIP(hipMemcpyAsync(m + at, t.start.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    at += a16(n * sizeof(int));
    d.count = (const int*)(m + at);
    SGMG_HIP(hipMemcpyAsync(m + at, t.count.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    at += a16(n * sizeof(int));
    dts.push_back(d);
  }
  at = bytes;
  st.part = (double*)(m + at);
  at += (part_b + 255) & ~(size_t)255;
  st.scal = (double*)(m + at);
  at += (scal_b + 255) & ~(size_t)255;
  st.flags = (int*)(m + at);
  int k = 0;
  st.tv = dts[k++];
  for (int l = 0; l < st.Lmax - 1; ++l) {
    st.ts[l] = dts[k++];
    st.tr[l] = dts[k++];
  }
  st.tcg = dts[k++];
  st.tcm = dts[k++];
  for (int l = 1; l < st.Lmax - 1; ++l) {
    st.tsc[l] = dts[k++];
    st.tss[l] = dts[k++];
  }
  BsTable k64t[kK64];
  if (mf64)
    for (int c = 0; c < kK64; ++c) k64t[c] = dts[k++];
  if (hipHostMalloc((void**)&st.h_flags, flag_b, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&st.h_scal, scal_b, hipHostMallocDefault) != hipSuccess) {
    set_error("staged batch host allocation failed");
    return SGMG_ENOMEM;
  }
  SGMG_HIP(hipStreamSynchronize(s));
  // level 0 on the matrix cores when every item's system runs its fine
  // level in BF16X3 on the MFMA operator
  bool mf = true;
  for (int i = 0; i < n; ++i) {
    const sgmg_hierarchy* h = b->hs[b->h_items[i].sys];
    mf = mf && h->L > 1 && h->lev[0].f32 && level_prec(h, 0) == SGMG_BF16X3 && h->kt.integral &&
         mfma_size_ok(h->lev[0].g);
  }
  st.mfma0 = mf;
  if (mf) TRY(bs_tune_mfma(b, n, s));
  TRY(bs_tune_stencil(b, n, s));
  if (mf64) {
    // per-item tile grids of each candidate shape; time the K p stage of
    // every item (three launches after one warm-up) and keep the fastest
    std::vector<int4> g64((size_t)kK64 * n);
    for (int c = 0; c < kK64; ++c)
      for (int i = 0; i < n; ++i)
        g64[(size_t)c * n + i] = bs_mfma_geometry(b->hs[b->h_items[i].sys]->lev[0].g,
                                                  geo_rows(k64_shapes[c][0]), k64_shapes[c][1]);
    if (hipMalloc(&st.m64dmem, g64.size() * sizeof(int4)) != hipSuccess) {
      set_error("staged batch allocation failed");
      return SGMG_ENOMEM;
    }
    int4* dg = (int4*)st.m64dmem;
    SGMG_HIP(hipMemcpyAsync(dg, g64.data(), g64.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    std::vector<int> ones(n, 1);
    SGMG_HIP(hipMemcpyAsync(st.flags, ones.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    hipEvent_t e0, e1;
    SGMG_HIP(hipEventCreate(&e0));
    SGMG_HIP(hipEventCreate(&e1));
    const BsArgs a{b->d_sys, b->d_items};
    float best = 0.f;
    int bc = -1;
    for (int c = 0; c < kK64; ++c) {
      const int4* gc = dg + (size_t)c * n;
      bs_fine_mfma64_store_dot(a, k64t[c], gc, st.flags, k64_shapes[c][0], k64_shapes[c][1], st.part, s);
      SGMG_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r)
        bs_fine_mfma64_store_dot(a, k64t[c], gc, st.flags, k64_shapes[c][0], k64_shapes[c][1], st.part, s);
      SGMG_HIP(hipEventRecord(e1, s));
      SGMG_HIP(hipEventSynchronize(e1));
      TRY(check_launch());
      float ms = 0.f;
      SGMG_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (bc < 0 || ms < best) { best = ms; bc = c; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    st.mfma64 = true;
    st.tk64 = k64t[bc];
    st.geo64 = dg + (size_t)bc * n;
    st.k64rows = k64_shapes[bc][0];
    st.k64z = k64_shapes[bc][1];
  }
  TRY(bs_capture(b, bs_prologue, n, &st.g_pro));
  TRY(bs_capture(b, bs_iteration, n, &st.g_it));
  st.ready = true;
  return 0;
}

}  // namespace

extern "C" {

void sgmg_batch_destroy(sgmg_batch* b) {
  if (!b) return;
  batch_free_items(b);
  for (sgmg_hierarchy* h : b->hs) sgmg_destroy(h);
  if (b->d_sys) hipFree(b->d_sys);
  if (b->d_queue) hipFree(b->d_queue);
  if (b->cap) hipStreamDestroy(b->cap);
  delete b;
}

int sgmg_setup_batch(int nsys, const sgmg_options* opts, const double* const* rho_or_E,
                     const uint8_t* const* fixed_dof, void* stream, sgmg_batch** out) {
  if (out) *out = nullptr;
  if (nsys < 1 || !opts || !rho_or_E || !out) { set_error("bad batch arguments"); return SGMG_EINVAL; }
  hipStream_t s = as_stream(stream);
  sgmg_batch* b = new (std::nothrow) sgmg_batch();
  if (!b) { set_error("host allocation failed"); return SGMG_ENOMEM; }
  for (int i = 0; i < nsys; ++i) {
    sgmg_hierarchy* h = nullptr;
    const int rc = sgmg_setup_hierarchy(&opts[i], rho_or_E[i], fixed_dof ? fixed_dof[i] : nullptr,
                                        stream, &h);
    if (rc) { sgmg_batch_destroy(b); return rc; }
    b->hs.push_back(h);
    if (h->coarse_iter) {
      sgmg_batch_destroy(b);
      set_error("batched systems need a dense coarsest solve (coarsest free DOFs <= dense_max)");
      return SGMG_EINVAL;
    }
    if (h->o.cycle_gamma != 1) {
      sgmg_batch_destroy(b);
      set_error("batched systems use the V-cycle (cycle_gamma 1)");
      return SGMG_EINVAL;
    }
  }
  std::vector<BSys> hsys;
  for (auto* h : b->hs) hsys.push_back(make_bsys(h));
  if (hipMalloc(&b->d_sys, hsys.size() * sizeof(BSys)) != hipSuccess ||
      hipMalloc(&b->d_queue, sizeof(int)) != hipSuccess) {
    sgmg_batch_destroy(b);
    set_error("batch allocation failed");
    return SGMG_ENOMEM;
  }
  hipMemcpyAsync(b->d_sys, hsys.data(), hsys.size() * sizeof(BSys), hipMemcpyHostToDevice, s);
  if (hipStreamSynchronize(s) != hipSuccess) { sgmg_batch_destroy(b); set_error("sync failed"); return SGMG_EHIP; }
  *out = b;
  return 0;
}

sgmg_hierarchy* sgmg_batch_hierarchy(sgmg_batch* b, int sys) {
  if (!b || sys < 0 || sys >= (int)b->hs.size()) return nullptr;
  return b->hs[sys];
}

int sgmg_batch_block_size(const sgmg_batch* b) { return b ? b->bs : 0; }

size_t sgmg_batch_item_layout(int L, const int* level_dofs, int nL, size_t* offsets,
                              size_t* sizes) {
  if (L < 2 || L > kMaxLevels || !level_dofs) return 0;
  for (int l = 0; l < L; ++l)
    if (level_dofs[l] < 1) return 0;
  // every sub-buffer starts on a 256-byte boundary: each one's size rounded
  auto rounded = [](size_t nbytes) { return (nbytes + 255) & ~(size_t)255; };
  size_t at = 0;
  int k = 0;
  auto take = [&](size_t nbytes) {
    if (offsets) offsets[k] = at;
    if (sizes) sizes[k] = nbytes;
    ++k;
    at += rounded(nbytes);
  };
  const size_t n0 = (size_t)level_dofs[0];
  for (int i = 0; i < 5; ++i) take(n0 * sizeof(double));    // r, z, p, q, t
  for (int i = 0; i < 5; ++i) take(n0 * sizeof(float));     // b0, d0, r0, x0[2]
  for (int l = 1; l < L; ++l)
    for (int i = 0; i < 4; ++i) take((size_t)level_dofs[l] * sizeof(double));   // b, x[2], r
  take((size_t)std::max(nL, 1) * sizeof(double));           // coarsest right-hand side
  return at;
}

int sgmg_pcg_solve_batch(sgmg_batch* b, int nitems, const int* item_sys, const double* const* f,
                         double* const* u, double rtol, int maxit, sgmg_solve_info* infos,
                         double* total_ms, void* stream) {
  if (!b || nitems < 1 || !item_sys || !f || !u || maxit < 0) { set_error("bad batch solve arguments"); return SGMG_EINVAL; }
  for (int i = 0; i < nitems; ++i)
    if (item_sys[i] < 0 || item_sys[i] >= (int)b->hs.size() || !f[i] || !u[i]) {
      set_error("bad item " + std::to_string(i));
      return SGMG_EINVAL;
    }
  hipStream_t s = as_stream(stream);
  TRY(batch_prepare_items(b, nitems, item_sys, s));
  for (int k = 0; k < nitems; ++k) {
    b->h_items[k].f = f[b->order[k]];
    b->h_items[k].u = u[b->order[k]];
  }
  SGMG_HIP(hipMemcpyAsync(b->d_items, b->h_items.data(), nitems * sizeof(BItem), hipMemcpyHostToDevice, s));
  if (b->bs == 0) {
    // autotune the block size on this batch (2 iterations per candidate), then restore u
    std::vector<double*> saved(nitems, nullptr);
    int rc = 0;
    for (int k = 0; k < nitems && !rc; ++k) {
      const size_t n = b->hs[b->h_items[k].sys]->lev[0].g.n;
      if (hipMalloc(&saved[k], n * sizeof(double)) != hipSuccess) { rc = SGMG_ENOMEM; break; }
      hipMemcpyAsync(saved[k], b->h_items[k].u, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    }
    float best = 1e30f;
    int best_bs = 256;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    for (int bs : {256, 512}) {
      if (rc) break;
      hipEventRecord(e0, s);
      launch_batch_pcg(bs, std::min(nitems, 1024), b->d_sys, b->d_items, nitems, b->d_queue,
                       b->d_out, rtol, 2, s);
      hipEventRecord(e1, s);
      if ((rc = check_launch())) break;
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; best_bs = bs; }
      for (int k = 0; k < nitems; ++k) {
        const size_t n = b->hs[b->h_items[k].sys]->lev[0].g.n;
        hipMemcpyAsync(b->h_items[k].u, saved[k], n * sizeof(double), hipMemcpyDeviceToDevice, s);
      }
    }
    hipStreamSynchronize(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    for (double* p : saved) if (p) hipFree(p);
    if (rc) return rc;
    b->bs = best_bs;
  }
  hipEvent_t e0, e1;
  SGMG_HIP(hipEventCreate(&e0));
  SGMG_HIP(hipEventCreate(&e1));
  SGMG_HIP(hipEventRecord(e0, s));
  const int rc = batch_launch(b, nitems, rtol, maxit, b->bs, s);
  if (rc) { hipEventDestroy(e0); hipEventDestroy(e1); return rc; }
  SGMG_HIP(hipEventRecord(e1, s));
  SGMG_HIP(hipMemcpyAsync(b->h_out, b->d_out, nitems * sizeof(BOut), hipMemcpyDeviceToHost, s));
  SGMG_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (total_ms) *total_ms = ms;
  if (infos) {
    for (int k = 0; k < nitems; ++k) {
      sgmg_solve_info& inf = infos[b->order[k]];
      inf.status = b->h_out[k].status;
      inf.iters = b->h_out[k].iters;
      inf.rel_res_true = b->h_out[k].rel_true;
      inf.rel_res_recur = b->h_out[k].rel_recur;
      inf.solve_ms = ms;
      inf.fallback_iter = -1;
    }
  }
  return 0;
}

int sgmg_pcg_solve_batch_staged(sgmg_batch* b, int nitems, const int* item_sys,
                                const double* const* f, double* const* u, double rtol, int maxit,
                                sgmg_solve_info* infos, double* total_ms, void* stream) {
  if (!b || nitems < 1 || !item_sys || !f || !u || maxit < 0 || !(rtol > 0.0)) {
    set_error("bad batch solve arguments");
    return SGMG_EINVAL;
  }
  for (int i = 0; i < nitems; ++i)
    if (item_sys[i] < 0 || item_sys[i] >= (int)b->hs.size() || !f[i] || !u[i]) {
      set_error("bad item " + std::to_string(i));
      return SGMG_EINVAL;
    }
  hipStream_t s = as_stream(stream);
  TRY(batch_prepare_items(b, nitems, item_sys, s));
  for (int k = 0; k < nitems; ++k) {
    b->h_items[k].f = f[b->order[k]];
    b->h_items[k].u = u[b->order[k]];
  }
  SGMG_HIP(hipMemcpyAsync(b->d_items, b->h_items.data(), nitems * sizeof(BItem), hipMemcpyHostToDevice, s));
  TRY(bs_prepare(b, nitems, s));
  auto& st = b->st;
  const int n = nitems;
  int* hf = st.h_flags;
  double* hs = st.h_scal;
  std::vector<int> status(n, -1), iters(n, 0);
  std::vector<double> nf(n, 0.0), rel(n, 0.0), rel_true(n, -1.0);
  hipEvent_t e0, e1;
  SGMG_HIP(hipEventCreate(&e0));
  SGMG_HIP(hipEventCreate(&e1));
  SGMG_HIP(hipEventRecord(e0, s));
  // one graph replay with the given prologue / iteration flags, then the scalars
  auto run = [&](hipGraphExec_t g) -> int {
    SGMG_HIP(hipMemcpyAsync(st.flags, hf, 2 * (size_t)n * sizeof(int), hipMemcpyHostToDevice, s));
    SGMG_HIP(hipGraphLaunch(g, s));
    SGMG_HIP(hipMemcpyAsync(hs, st.scal, (size_t)n * kBsScalars * sizeof(double), hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipStreamSynchronize(s));
    return 0;
  };
  auto sc = [&](int i, int k) { return hs[(size_t)i * kBsScalars + k]; };
  // prologue for every item: true residual from x0, first V-cycle
  for (int i = 0; i < n; ++i) { hf[i] = 1; hf[n + i] = 0; }
  TRY(run(st.g_pro));
  for (int i = 0; i < n; ++i) {
    nf[i] = std::sqrt(sc(i, kBsFF));
    if (nf[i] == 0.0) {
      // f = 0: the solution is u = 0
      const size_t nn = b->hs[b->h_items[i].sys]->lev[0].g.n;
      SGMG_HIP(hipMemsetAsync(b->h_items[i].u, 0, nn * sizeof(double), s));
      status[i] = SGMG_CONVERGED;
      rel[i] = rel_true[i] = 0.0;
      continue;
    }
    rel[i] = std::sqrt(sc(i, kBsRR)) / nf[i];
    if (!std::isfinite(rel[i])) { status[i] = SGMG_NONFINITE; continue; }
    if (rel[i] < rtol) { status[i] = SGMG_CONVERGED; rel_true[i] = rel[i]; continue; }
    if (maxit == 0) { status[i] = SGMG_MAXIT; continue; }
    const double rz = sc(i, kBsRZ);
    if (!std::isfinite(rz)) { status[i] = SGMG_NONFINITE; continue; }
    if (rz <= 0.0) { status[i] = SGMG_BREAKDOWN; continue; }
  }
  for (int it = 1; it <= maxit; ++it) {
    int nact = 0;
    for (int i = 0; i < n; ++i) {
      hf[i] = 0;
      hf[n + i] = status[i] < 0;
      nact += hf[n + i];
    }
    if (!nact) break;
    TRY(run(st.g_it));
    int ncheck = 0;
    for (int i = 0; i < n; ++i) {
      hf[n + i] = 0;
      if (status[i] >= 0) continue;
      iters[i] = it;
      const double pq = sc(i, kBsPQ);
      if (!std::isfinite(pq)) { status[i] = SGMG_NONFINITE; iters[i] = it - 1; continue; }
      if (pq <= 0.0) { status[i] = SGMG_BREAKDOWN; iters[i] = it - 1; continue; }
      rel[i] = std::sqrt(sc(i, kBsRR)) / nf[i];
      if (!std::isfinite(rel[i])) { status[i] = SGMG_NONFINITE; continue; }
      if (rel[i] < rtol) { hf[i] = 1; ++ncheck; continue; }   // true-residual check
      const double rz = sc(i, kBsRZNew);
      if (!std::isfinite(rz)) { status[i] = SGMG_NONFINITE; continue; }
      if (rz <= 0.0) { status[i] = SGMG_BREAKDOWN; continue; }
      if (it == maxit) status[i] = SGMG_MAXIT;
    }
    if (ncheck) {
      // the prologue recomputes r = f - K x in FP64 and restarts the
      // recurrence from it (beta = 0) for the items that continue
      TRY(run(st.g_pro));
      for (int i = 0; i < n; ++i) {
        if (!hf[i]) continue;
        const double rt = std::sqrt(sc(i, kBsRR)) / nf[i];
        if (rt < rtol) { status[i] = SGMG_CONVERGED; rel_true[i] = rt; continue; }
        rel[i] = rt;
        const double rz = sc(i, kBsRZ);
        if (!std::isfinite(rz)) status[i] = SGMG_NONFINITE;
        else if (rz <= 0.0) status[i] = SGMG_BREAKDOWN;
        else if (it == maxit) status[i] = SGMG_MAXIT;
      }
    }
  }
  // true residual of the items that stopped without one
  int nleft = 0;
  for (int i = 0; i < n; ++i) {
    if (status[i] < 0) status[i] = SGMG_MAXIT;
    hf[i] = rel_true[i] < 0.0;
    hf[n + i] = 0;
    nleft += hf[i];
  }
  if (nleft) {
    TRY(run(st.g_pro));
    for (int i = 0; i < n; ++i)
      if (hf[i]) rel_true[i] = std::sqrt(sc(i, kBsRR)) / (nf[i] > 0.0 ? nf[i] : 1.0);
  }
  SGMG_HIP(hipEventRecord(e1, s));
  SGMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (total_ms) *total_ms = ms;
  if (infos) {
    for (int k = 0; k < n; ++k) {
      sgmg_solve_info& inf = infos[b->order[k]];
      inf.status = status[k];
      inf.iters = iters[k];
      inf.rel_res_true = rel_true[k];
      inf.rel_res_recur = rel[k];
      inf.solve_ms = ms;
      inf.fallback_iter = -1;
    }
  }
  return 0;
}

int sgmg_pcg_solve_batch_graph(sgmg_batch* b, int nitems, const int* item_sys,
                               const double* const* f, double* const* u, double rtol, int maxit,
                               int steps, sgmg_solve_info* infos, int* launches, double* total_ms,
                               void* stream) {
  if (!b || nitems < 1 || !item_sys || !f || !u || maxit < 0 || !(rtol > 0.0) || steps < 2 ||
      steps > 1024 || (steps & 1)) {
    set_error("bad batch solve arguments");
    return SGMG_EINVAL;
  }
  for (int i = 0; i < nitems; ++i)
    if (item_sys[i] < 0 || item_sys[i] >= (int)b->hs.size() || !f[i] || !u[i]) {
      set_error("bad item " + std::to_string(i));
      return SGMG_EINVAL;
    }
  hipStream_t s = as_stream(stream);
  TRY(batch_prepare_items(b, nitems, item_sys, s));
  for (int k = 0; k < nitems; ++k) {
    b->h_items[k].f = f[b->order[k]];
    b->h_items[k].u = u[b->order[k]];
  }
  SGMG_HIP(hipMemcpyAsync(b->d_items, b->h_items.data(), nitems * sizeof(BItem), hipMemcpyHostToDevice, s));
  TRY(bs_prepare(b, nitems, s));
  TRY(bs_prepare_loop(b, nitems, rtol, maxit, steps, s));
  auto& st = b->st;
  const int n = nitems;
  const int* hst = (const int*)st.h_lmem;           // the mirror of st.lp
  const size_t ib = (const char*)st.lp.nf - (const char*)st.lmem;
  const double* hd = (const double*)((const char*)st.h_lmem + ib);
  hipEvent_t e0, e1;
  SGMG_HIP(hipEventCreate(&e0));
  SGMG_HIP(hipEventCreate(&e1));
  SGMG_HIP(hipEventRecord(e0, s));
  // one launch covers steps iterations; another follows only while an item
  // still iterates after them
  int nl = 0;
  for (;;) {
    const hipError_t e = hipGraphLaunch(nl ? st.g_more : st.g_first, s);
    if (e != hipSuccess) {
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      set_error(std::string("batch loop launch: ") + hipGetErrorString(e));
      return SGMG_EHIP;
    }
    ++nl;
    SGMG_HIP(hipMemcpyAsync(st.h_lmem, st.lmem, st.lbytes, hipMemcpyDeviceToHost, s));
    SGMG_HIP(hipStreamSynchronize(s));
    bool active = false;
    for (int i = 0; i < n; ++i) active = active || hst[i] < 0;
    if (!active) break;
  }
  SGMG_HIP(hipEventRecord(e1, s));
  SGMG_HIP(hipEventSynchronize(e1));
  TRY(check_launch());
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (total_ms) *total_ms = ms;
  if (launches) *launches = nl;
  if (infos) {
    for (int k = 0; k < n; ++k) {
      sgmg_solve_info& inf = infos[b->order[k]];
      inf.status = hst[k];
      inf.iters = hst[n + k];
      inf.rel_res_true = hd[2 * n + k];
      inf.rel_res_recur = hd[n + k];
      inf.solve_ms = ms;
      inf.fallback_iter = -1;
    }
  }
  return 0;
}

int sgmg_pcg_solve_batch_concurrent(sgmg_batch* b, int nitems, const int* item_sys,
                                    const double* const* f, double* const* u, double rtol,
                                    int maxit, int nworkers, sgmg_solve_info* infos,
                                    double* total_ms, void* stream) {
  if (!b || nitems < 1 || !item_sys || !f || !u || maxit < 0 || nworkers < 1 || nworkers > 16) {
    set_error("bad batch solve arguments");
    return SGMG_EINVAL;
  }
  const int nsys = (int)b->hs.size();
  std::vector<std::vector<int>> by_sys(nsys);
  for (int i = 0; i < nitems; ++i) {
    if (item_sys[i] < 0 || item_sys[i] >= nsys || !f[i] || !u[i]) {
      set_error("bad item " + std::to_string(i));
      return SGMG_EINVAL;
    }
    by_sys[item_sys[i]].push_back(i);
  }
  // systems largest work first (DOFs x load cases), so the long solves start
  // first and the short ones fill the tail
  std::vector<int> order;
  for (int k = 0; k < nsys; ++k)
    if (!by_sys[k].empty()) order.push_back(k);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return (double)b->hs[a]->lev[0].g.n * by_sys[a].size() >
           (double)b->hs[c]->lev[0].g.n * by_sys[c].size();
  });
  int dev = 0;
  SGMG_HIP(hipGetDevice(&dev));
  // Every system's iteration graphs are captured here, on the calling
  // thread, before any worker starts (sgmg_set_launch_shape drops them): the
  // workers only launch graphs and never capture concurrently.
  for (int k : order) TRY(capture_vcycle_graphs(b->hs[k], as_stream(stream)));
  SGMG_HIP(hipStreamSynchronize(as_stream(stream)));   // the inputs are ready
  std::atomic<int> next{0};
  std::atomic<int> failed{0};
  std::mutex mu;
  std::string first_err;
  auto worker = [&]() {
    if (hipSetDevice(dev) != hipSuccess) { failed = SGMG_EHIP; return; }
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      std::lock_guard<std::mutex> lk(mu);
      if (!failed) { failed = SGMG_EHIP; first_err = "worker stream creation failed"; }
      return;
    }
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= (int)order.size() || failed) break;
      sgmg_hierarchy* h = b->hs[order[k]];
      for (int i : by_sys[order[k]]) {      // one system's load cases in order
        sgmg_solve_info local{};
        sgmg_solve_info* inf = infos ? &infos[i] : &local;
        const int rc = sgmg_pcg_solve(h, 2, f[i], u[i], rtol, maxit, inf, st);
        if (rc) {
          std::lock_guard<std::mutex> lk(mu);
          if (!failed) { failed = rc; first_err = sgmg_last_error(); }
          break;
        }
      }
    }
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  };
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<std::thread> pool;
  const int nw = std::min<int>(nworkers, (int)order.size());
  for (int w = 0; w < nw; ++w) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (total_ms) *total_ms = ms;
  if (failed) {
    set_error(first_err.empty() ? "concurrent batch solve failed" : first_err);
    return failed;
  }
  return 0;
}

int sgmg_level_info(const sgmg_hierarchy* h, int level, int* dims, int* n_free, double* lambda) {
  if (!h || level < 0 || level >= h->L) { set_error("bad level"); return SGMG_EINVAL; }
  const Level& L = h->lev[level];
  if (dims) { dims[0] = L.g.nx; dims[1] = L.g.ny; dims[2] = L.g.nz; }
  if (n_free) *n_free = L.n_free;
  if (lambda) *lambda = L.lam;
  return 0;
}

int sgmg_copy_stencil(const sgmg_hierarchy* h, int level, double* host_out) {
  if (!h || level < 1 || level >= h->L || !host_out) { set_error("bad level"); return SGMG_EINVAL; }
  const Level& L = h->lev[level];
  SGMG_HIP(hipMemcpy(host_out, L.S64, (size_t)kStencil * L.g.Nn * sizeof(double),
                     hipMemcpyDeviceToHost));
  return 0;
}

int sgmg_copy_diagonal(const sgmg_hierarchy* h, int level, double* host_out) {
  if (!h || level < 0 || level >= h->L || !host_out) { set_error("bad level"); return SGMG_EINVAL; }
  const Level& L = h->lev[level];
  SGMG_HIP(hipMemcpy(host_out, L.d64, (size_t)L.g.n * sizeof(double), hipMemcpyDeviceToHost));
  return 0;
}

// ---------------------------------------------------------------------------
// SIMP outer loop (Sec. 3.1, Eq. simp_filter; Sec. 3.5 drift rule through
// sgmg_update_moduli).
}  // extern "C"

struct sgmg_simp {
  sgmg_simp_params p{};
  double* W = nullptr;       // filter row sums
  double* rhohat = nullptr;
  double* dH = nullptr;
  double* gc = nullptr;      // dH * dc/drhohat
  double* ratio = nullptr;   // OC ratio max(-dc, 0) / dv
  RedWs ws{};
  double* sc = nullptr;      // [0] compliance, [1] volume
  double* h_sc = nullptr;
  std::vector<double> h_part;
  bool have_physical = false, have_ratio = false;
  std::vector<void*> allocs;
};

namespace {

int simp_alloc(sgmg_simp* s, double** p, size_t count) {
  void* v = nullptr;
  if (hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(double)) != hipSuccess) {
    set_error("SIMP allocation failed");
    return SGMG_ENOMEM;
  }
  s->allocs.push_back(v);
  *p = (double*)v;
  return 0;
}

}  // namespace

extern "C" {

void sgmg_simp_default_params(sgmg_simp_params* p, int nx, int ny, int nz) {
  std::memset(p, 0, sizeof(*p));
  p->nx = nx; p->ny = ny; p->nz = nz;
  p->penal = 3.0; p->E0 = 1.0; p->Emin = 1e-9;
  p->volfrac = 0.5; p->move = 0.2;
  p->rmin = 1.5; p->beta = 0.0; p->eta = 0.5;
  p->oc_tol = 1e-9; p->oc_max_halvings = 200;
}

void sgmg_simp_destroy(sgmg_simp* s) {
  if (!s) return;
  for (void* v : s->allocs) hipFree(v);
  if (s->h_sc) hipHostFree(s->h_sc);
  delete s;
}

int sgmg_simp_create(const sgmg_simp_params* p, void* stream, sgmg_simp** out) {
  if (out) *out = nullptr;
  if (!p || !out) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || (long)p->nx * p->ny * p->nz > 0x7fffffffL) {
    set_error("bad SIMP mesh"); return SGMG_EINVAL;
  }
  if (!(p->rmin > 0.0) || p->rmin > 16.0 || !(p->volfrac > 0.0 && p->volfrac < 1.0) ||
      !(p->move > 0.0) || !(p->beta >= 0.0) || !(p->eta > 0.0 && p->eta < 1.0) ||
      !(p->penal >= 1.0) || !(p->oc_tol > 0.0) || p->oc_max_halvings < 1) {
    set_error("bad SIMP parameters"); return SGMG_EINVAL;
  }
  sgmg_simp* s = new (std::nothrow) sgmg_simp();
  if (!s) { set_error("host allocation failed"); return SGMG_ENOMEM; }
  s->p = *p;
  const size_t n = (size_t)p->nx * p->ny * p->nz;
  const size_t nb = div_up((int)n, 256) + 2048;
  int rc = 0;
  if ((rc = simp_alloc(s, &s->W, n)) || (rc = simp_alloc(s, &s->rhohat, n)) ||
      (rc = simp_alloc(s, &s->dH, n)) || (rc = simp_alloc(s, &s->gc, n)) ||
      (rc = simp_alloc(s, &s->ratio, n)) || (rc = simp_alloc(s, &s->ws.partials, nb)) ||
      (rc = simp_alloc(s, &s->sc, 4))) {
    sgmg_simp_destroy(s);
    return rc;
  }
  if (hipHostMalloc((void**)&s->h_sc, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    sgmg_simp_destroy(s);
    set_error("pinned allocation failed");
    return SGMG_ENOMEM;
  }
  hipStream_t st = as_stream(stream);
  launch_filter_wsum(p->nx, p->ny, p->nz, p->rmin, s->W, st);
  if ((rc = check_launch()) || hipStreamSynchronize(st) != hipSuccess) {
    sgmg_simp_destroy(s);
    if (!rc) { set_error("sync failed"); rc = SGMG_EHIP; }
    return rc;
  }
  *out = s;
  return 0;
}

int sgmg_simp_physical(sgmg_simp* s, const double* rho, double* rhohat, void* stream) {
  if (!s || !rho) { set_error("NULL argument"); return SGMG_EINVAL; }
  hipStream_t st = as_stream(stream);
  const sgmg_simp_params& p = s->p;
  launch_physical(p.nx, p.ny, p.nz, p.rmin, s->W, rho, p.beta, p.eta, s->rhohat, s->dH, st);
  TRY(check_launch());
  if (rhohat)
    SGMG_HIP(hipMemcpyAsync(rhohat, s->rhohat, (size_t)p.nx * p.ny * p.nz * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
  s->have_physical = true;
  s->have_ratio = false;
  return 0;
}

int sgmg_simp_sensitivity(sgmg_simp* s, const sgmg_hierarchy* h, const double* u,
                          double* compliance, double* dc, double* dv, void* stream) {
  if (!s || !h || !u) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (!s->have_physical) { set_error("sgmg_simp_physical must run first"); return SGMG_EINVAL; }
  const sgmg_simp_params& p = s->p;
  const Grid& g = h->lev[0].g;
  if (g.nx != p.nx || g.ny != p.ny || g.nz != p.nz) { set_error("hierarchy mesh differs"); return SGMG_EINVAL; }
  hipStream_t st = as_stream(stream);
  launch_element_energy(g, h->ke64, s->rhohat, s->dH, u, p.penal, p.E0, p.Emin, s->gc, s->ws,
                        s->sc, st);
  launch_oc_ratio(p.nx, p.ny, p.nz, p.rmin, s->W, s->gc, s->dH, s->ratio, dc, dv, st);
  TRY(check_launch());
  SGMG_HIP(hipMemcpyAsync(s->h_sc, s->sc, sizeof(double), hipMemcpyDeviceToHost, st));
  SGMG_HIP(hipStreamSynchronize(st));
  if (compliance) *compliance = s->h_sc[0];
  s->have_ratio = true;
  return 0;
}

int sgmg_simp_oc_update(sgmg_simp* s, double* rho, double* lambda, double* volume,
                        double* max_change, void* stream) {
  if (!s || !rho) { set_error("NULL argument"); return SGMG_EINVAL; }
  if (!s->have_ratio) { set_error("sgmg_simp_sensitivity must run first"); return SGMG_EINVAL; }
  const sgmg_simp_params& p = s->p;
  const int n = p.nx * p.ny * p.nz;
  const double target = p.volfrac * n;
  hipStream_t st = as_stream(stream);
  double l1 = 0.0, l2 = 1e9, lmid = 0.5 * (l1 + l2), vol = 0.0;
  for (int it = 0; it < p.oc_max_halvings; ++it) {
    lmid = 0.5 * (l1 + l2);
    launch_oc_volume(p.nx, p.ny, p.nz, p.rmin, s->W, rho, s->ratio, lmid, p.move, p.beta, p.eta,
                     s->ws, s->sc + 1, st);
    TRY(check_launch());
    SGMG_HIP(hipMemcpyAsync(s->h_sc + 1, s->sc + 1, sizeof(double), hipMemcpyDeviceToHost, st));
    SGMG_HIP(hipStreamSynchronize(st));
    vol = s->h_sc[1];
    if (!std::isfinite(vol)) { set_error("OC volume is not finite"); return SGMG_EINVAL; }
    if (vol > target) l1 = lmid;
    else l2 = lmid;
    if (l2 - l1 <= p.oc_tol * (l1 + l2)) break;
  }
  launch_oc_apply(n, rho, s->ratio, lmid, p.move, s->ws, st);
  TRY(check_launch());
  const int nb = oc_apply_blocks(n);
  s->h_part.resize(nb);
  SGMG_HIP(hipMemcpyAsync(s->h_part.data(), s->ws.partials, nb * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  SGMG_HIP(hipStreamSynchronize(st));
  double m = 0.0;
  for (double v : s->h_part) m = std::max(m, v);
  if (lambda) *lambda = lmid;
  if (volume) *volume = vol;
  if (max_change) *max_change = m;
  s->have_physical = s->have_ratio = false;
  return 0;
}

int sgmg_simp_step(sgmg_simp* s, sgmg_hierarchy* h, int precond, double* rho, const double* f,
                   double* u, double rtol, int maxit, sgmg_simp_info* info, void* stream) {
  if (!s || !h || !rho || !f || !u) { set_error("NULL argument"); return SGMG_EINVAL; }
  const sgmg_simp_params& p = s->p;
  const sgmg_options& o = h->o;
  if (o.input_is_modulus || o.penal != p.penal || o.E0 != p.E0 || o.Emin != p.Emin) {
    set_error("hierarchy SIMP map (input_is_modulus 0, penal, E0, Emin) differs from the SIMP parameters");
    return SGMG_EINVAL;
  }
  TRY(sgmg_simp_physical(s, rho, nullptr, stream));
  TRY(sgmg_update_moduli(h, s->rhohat, stream));
  sgmg_solve_info si{};
  TRY(sgmg_pcg_solve(h, precond, f, u, rtol, maxit, &si, stream));
  double c = 0.0, lam = 0.0, vol = 0.0, chg = 0.0;
  TRY(sgmg_simp_sensitivity(s, h, u, &c, nullptr, nullptr, stream));
  TRY(sgmg_simp_oc_update(s, rho, &lam, &vol, &chg, stream));
  if (info) {
    info->compliance = c;
    info->volume = vol;
    info->lambda = lam;
    info->max_change = chg;
    info->pcg_status = si.status;
    info->pcg_iters = si.iters;
    info->rel_res_true = si.rel_res_true;
    info->solve_ms = si.solve_ms;
  }
  return 0;
}

}  // extern "C"
