// Warm-start U-Net: parameters, forward, backward, Adam, and the C ABI
// (extension; see include/simpgmg.h for the network description).
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "unet.hpp"

using namespace sgmg;

namespace {

constexpr int kNL = 8;
const int kCi[kNL] = {5, 16, 32, 64, 128, 64, 32, 16};
const int kCo[kNL] = {16, 32, 64, 128, 64, 32, 16, 3};
const int kK[kNL] = {3, 3, 3, 3, 3, 3, 3, 1};

int pad16(int c) { return (c + 15) / 16 * 16; }

struct ULayer {
  int ci, co, k, k3, cop, cip;
  size_t nw;                  // ci * k3 * cop
  float *w, *wq, *b, *gw, *gb, *mw, *vw, *mb, *vb, *wt;
};

}  // namespace

struct sgmg_unet {
  ULayer L[kNL];
  std::vector<void*> mem;
  int step = 0;
  // activation workspace for one (N, D, H, W)
  int aN = 0, aD = 0, aH = 0, aW = 0;
  std::vector<void*> act;
  float *r1 = nullptr, *p1, *r2, *p2, *r3, *p3, *r4, *u4, *r5, *d3, *u3, *r6, *d2, *u2, *r7, *d1,
        *y, *gy, *g1, *g2, *g3, *g4, *g5, *part;
  double* sums = nullptr;
  double* partials = nullptr;
  double h_sums[2];
};

namespace {

void set_err(const std::string& m) { sgmg::set_error(m); }

int ualloc(std::vector<void*>& mem, float** p, size_t n) {
  void* v = nullptr;
  if (hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(float)) != hipSuccess) {
    set_err("U-Net allocation failed");
    return SGMG_ENOMEM;
  }
  hipMemset(v, 0, std::max<size_t>(n, 1) * sizeof(float));
  mem.push_back(v);
  *p = (float*)v;
  return 0;
}

void free_act(sgmg_unet* u) {
  for (void* p : u->act) hipFree(p);
  u->act.clear();
  u->aN = 0;
}

int ensure_act(sgmg_unet* u, int N, int D, int H, int W) {
  if (u->aN == N && u->aD == D && u->aH == H && u->aW == W) return 0;
  free_act(u);
  const size_t v1 = (size_t)D * H * W, v2 = v1 / 8, v3 = v2 / 8, v4 = v3 / 8;
  struct Req { float** p; size_t n; };
  size_t part = 0;
  // input resolution of each conv (for the weight-gradient workspace)
  const int Dl[kNL] = {D, D / 2, D / 4, D / 8, D / 4, D / 2, D, D};
  const int Hl[kNL] = {H, H / 2, H / 4, H / 8, H / 4, H / 2, H, H};
  const int Wl[kNL] = {W, W / 2, W / 4, W / 8, W / 4, W / 2, W, W};
  for (int l = 0; l < kNL; ++l)
    part = std::max(part, conv_wgrad_part_floats(N, kCi[l], kCo[l], Dl[l], Hl[l], Wl[l], kK[l]));
  const Req reqs[] = {
      {&u->r1, N * 16 * v1}, {&u->p1, N * 16 * v2}, {&u->r2, N * 32 * v2}, {&u->p2, N * 32 * v3},
      {&u->r3, N * 64 * v3}, {&u->p3, N * 64 * v4}, {&u->r4, N * 128 * v4}, {&u->u4, N * 128 * v3},
      {&u->r5, N * 64 * v3}, {&u->d3, N * 64 * v3}, {&u->u3, N * 64 * v2}, {&u->r6, N * 32 * v2},
      {&u->d2, N * 32 * v2}, {&u->u2, N * 32 * v1}, {&u->r7, N * 16 * v1}, {&u->d1, N * 16 * v1},
      {&u->y, N * 3 * v1}, {&u->gy, N * 3 * v1}, {&u->g1, N * 128 * v1 / 4},
      {&u->g2, N * 128 * v1 / 4}, {&u->g3, N * 128 * v1 / 4}, {&u->g4, N * 128 * v1 / 4},
      {&u->g5, N * 128 * v1 / 4}, {&u->part, part}};
  // every activation/gradient buffer is sized for the largest tensor
  // (N x 32 x full resolution) so the backward pass can reuse them freely
  for (const Req& r : reqs)
    if (ualloc(u->act, r.p, std::max(r.n, (size_t)N * 32 * v1))) return SGMG_ENOMEM;
  void* s = nullptr;
  if (hipMalloc(&s, 2 * sizeof(double)) != hipSuccess) return SGMG_ENOMEM;
  u->act.push_back(s);
  u->sums = (double*)s;
  void* pp = nullptr;
  if (hipMalloc(&pp, 2 * 1024 * sizeof(double)) != hipSuccess) return SGMG_ENOMEM;
  u->act.push_back(pp);
  u->partials = (double*)pp;
  u->aN = N; u->aD = D; u->aH = H; u->aW = W;
  return 0;
}

// SplitMix64 normal draws (Box-Muller) for He initialisation.
double sm64_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((z >> 11) + 0.5) * 0x1.0p-53;
}

int check() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { set_err(std::string("U-Net kernel: ") + hipGetErrorString(e)); return SGMG_EHIP; }
  return 0;
}

void upload_layer(const ULayer& L, const std::vector<float>& w_dev_layout, const float* b, hipStream_t s) {
  hipMemcpyAsync(L.w, w_dev_layout.data(), L.nw * sizeof(float), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(L.b, b, L.co * sizeof(float), hipMemcpyHostToDevice, s);
  launch_round_bf16(L.w, L.wq, (long)L.nw, s);
}

void forward(sgmg_unet* u, int N, int D, int H, int W, const float* x, hipStream_t s) {
  const ULayer* L = u->L;
  const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4, D4 = D / 8,
            H4 = H / 8, W4 = W / 8;
  launch_conv_fwd(3, x, N, 5, 16, D, H, W, L[0].wq, L[0].b, 1, nullptr, nullptr, u->r1, s);
  launch_pool(u->r1, N * 16, D, H, W, u->p1, s);
  launch_conv_fwd(3, u->p1, N, 16, 32, D2, H2, W2, L[1].wq, L[1].b, 1, nullptr, nullptr, u->r2, s);
  launch_pool(u->r2, N * 32, D2, H2, W2, u->p2, s);
  launch_conv_fwd(3, u->p2, N, 32, 64, D3, H3, W3, L[2].wq, L[2].b, 1, nullptr, nullptr, u->r3, s);
  launch_pool(u->r3, N * 64, D3, H3, W3, u->p3, s);
  launch_conv_fwd(3, u->p3, N, 64, 128, D4, H4, W4, L[3].wq, L[3].b, 1, nullptr, nullptr, u->r4, s);
  launch_expand(u->r4, N * 128, D3, H3, W3, 1.f, u->u4, s);
  launch_conv_fwd(3, u->u4, N, 128, 64, D3, H3, W3, L[4].wq, L[4].b, 1, u->r5, u->r3, u->d3, s);
  launch_expand(u->d3, N * 64, D2, H2, W2, 1.f, u->u3, s);
  launch_conv_fwd(3, u->u3, N, 64, 32, D2, H2, W2, L[5].wq, L[5].b, 1, u->r6, u->r2, u->d2, s);
  launch_expand(u->d2, N * 32, D, H, W, 1.f, u->u2, s);
  launch_conv_fwd(3, u->u2, N, 32, 16, D, H, W, L[6].wq, L[6].b, 1, u->r7, u->r1, u->d1, s);
  launch_conv_fwd(1, u->d1, N, 16, 3, D, H, W, L[7].wq, L[7].b, 0, nullptr, nullptr, u->y, s);
}

// dx = data gradient of layer l (transposed, flipped weights)
void conv_dgrad(sgmg_unet* u, int l, const float* dy, int N, int D, int H, int W, float* dx,
                hipStream_t s) {
  const ULayer& L = u->L[l];
  launch_weight_transpose(L.wq, L.ci, L.co, L.k, L.wt, s);
  launch_conv_fwd(L.k, dy, N, L.co, L.ci, D, H, W, L.wt, nullptr, 0, nullptr, nullptr, dx, s);
}

void backward(sgmg_unet* u, int N, int D, int H, int W, const float* x, hipStream_t s) {
  const ULayer* L = u->L;
  const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4, D4 = D / 8,
            H4 = H / 8, W4 = W / 8;
  const long v1 = (long)D * H * W, v2 = v1 / 8, v3 = v2 / 8, v4 = v3 / 8;
  float *gd1 = u->g1, *gt = u->g2, *gd2 = u->g3, *gd3 = u->g4, *gt2 = u->g5;
  // output 1x1 conv
  launch_conv_wgrad(1, u->d1, u->gy, N, 16, 3, D, H, W, u->part, L[7].gw, L[7].gb, s);
  conv_dgrad(u, 7, u->gy, N, D, H, W, gd1, s);                       // dL/d d1 (skip to e1 too)
  launch_relu_bwd(gd1, u->r7, nullptr, N * 16 * v1, gt, s);          // dL/d r7 pre
  launch_conv_wgrad(3, u->u2, gt, N, 32, 16, D, H, W, u->part, L[6].gw, L[6].gb, s);
  conv_dgrad(u, 6, gt, N, D, H, W, gt2, s);                          // dL/d u2 [N,32,D]
  launch_sum8(gt2, N * 32, D, H, W, gd2, s);                         // dL/d d2 [N,32,D2]
  launch_relu_bwd(gd2, u->r6, nullptr, N * 32 * v2, gt, s);
  launch_conv_wgrad(3, u->u3, gt, N, 64, 32, D2, H2, W2, u->part, L[5].gw, L[5].gb, s);
  conv_dgrad(u, 5, gt, N, D2, H2, W2, gt2, s);                       // dL/d u3 [N,64,D2]
  launch_sum8(gt2, N * 64, D2, H2, W2, gd3, s);                      // dL/d d3 [N,64,D3]
  launch_relu_bwd(gd3, u->r5, nullptr, N * 64 * v3, gt, s);
  launch_conv_wgrad(3, u->u4, gt, N, 128, 64, D3, H3, W3, u->part, L[4].gw, L[4].gb, s);
  conv_dgrad(u, 4, gt, N, D3, H3, W3, gt2, s);                       // dL/d u4 [N,128,D3]
  launch_sum8(gt2, N * 128, D3, H3, W3, gt, s);                      // dL/d r4 [N,128,D4]
  launch_relu_bwd(gt, u->r4, nullptr, N * 128 * v4, gt2, s);
  launch_conv_wgrad(3, u->p3, gt2, N, 64, 128, D4, H4, W4, u->part, L[3].gw, L[3].gb, s);
  conv_dgrad(u, 3, gt2, N, D4, H4, W4, gt, s);                       // dL/d p3 [N,64,D4]
  launch_expand(gt, N * 64, D3, H3, W3, 0.125f, gt2, s);             // pool adjoint
  launch_relu_bwd(gt2, u->r3, gd3, N * 64 * v3, gt, s);              // + skip from d3
  launch_conv_wgrad(3, u->p2, gt, N, 32, 64, D3, H3, W3, u->part, L[2].gw, L[2].gb, s);
  conv_dgrad(u, 2, gt, N, D3, H3, W3, gt2, s);                       // dL/d p2 [N,32,D3]
  launch_expand(gt2, N * 32, D2, H2, W2, 0.125f, gt, s);
  launch_relu_bwd(gt, u->r2, gd2, N * 32 * v2, gt2, s);              // + skip from d2
  launch_conv_wgrad(3, u->p1, gt2, N, 16, 32, D2, H2, W2, u->part, L[1].gw, L[1].gb, s);
  conv_dgrad(u, 1, gt2, N, D2, H2, W2, gt, s);                       // dL/d p1 [N,16,D2]
  launch_expand(gt, N * 16, D, H, W, 0.125f, gt2, s);
  launch_relu_bwd(gt2, u->r1, gd1, N * 16 * v1, gt, s);              // + skip from d1
  launch_conv_wgrad(3, x, gt, N, 5, 16, D, H, W, u->part, L[0].gw, L[0].gb, s);
}

int check_dims(int N, int D, int H, int W) {
  if (N < 1 || D < 8 || H < 8 || W < 8 || D % 8 || H % 8 || W % 8) {
    set_err("U-Net volume must be N >= 1 and D, H, W multiples of 8 (>= 8)");
    return SGMG_EINVAL;
  }
  return 0;
}

}  // namespace

extern "C" {

void sgmg_unet_destroy(sgmg_unet* u) {
  if (!u) return;
  free_act(u);
  for (void* p : u->mem) hipFree(p);
  delete u;
}

int sgmg_unet_create(uint64_t seed, sgmg_unet** out) {
  if (!out) { set_err("NULL argument"); return SGMG_EINVAL; }
  *out = nullptr;
  sgmg_unet* u = new (std::nothrow) sgmg_unet();
  if (!u) { set_err("host allocation failed"); return SGMG_ENOMEM; }
  uint64_t ctr = 0;
  for (int l = 0; l < kNL; ++l) {
    ULayer& L = u->L[l];
    L.ci = kCi[l]; L.co = kCo[l]; L.k = kK[l]; L.k3 = L.k * L.k * L.k;
    L.cop = pad16(L.co); L.cip = pad16(L.ci);
    L.nw = (size_t)L.ci * L.k3 * L.cop;
    int rc = 0;
    for (float** p : {&L.w, &L.wq, &L.gw, &L.mw, &L.vw})
      if (!rc) rc = ualloc(u->mem, p, L.nw);
    for (float** p : {&L.b, &L.gb, &L.mb, &L.vb})
      if (!rc) rc = ualloc(u->mem, p, L.cop);
    if (!rc) rc = ualloc(u->mem, &L.wt, (size_t)L.co * L.k3 * L.cip);
    if (rc) { sgmg_unet_destroy(u); return rc; }
    // He-normal initialisation, zero bias, device layout [ci][tap][cop]
    std::vector<float> w(L.nw, 0.f), b(L.co, 0.f);
    const double sd = std::sqrt(2.0 / (L.ci * L.k3));
    for (int co = 0; co < L.co; ++co)
      for (int ci = 0; ci < L.ci; ++ci)
        for (int t = 0; t < L.k3; ++t) {
          const double u1 = sm64_uniform(seed, ctr++), u2 = sm64_uniform(seed, ctr++);
          const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
          w[((size_t)ci * L.k3 + t) * L.cop + co] = (float)(sd * z);
        }
    upload_layer(L, w, b.data(), 0);
  }
  if (hipDeviceSynchronize() != hipSuccess || check()) { sgmg_unet_destroy(u); return SGMG_EHIP; }
  *out = u;
  return 0;
}

int sgmg_unet_num_params(void) {
  int n = 0;
  for (int l = 0; l < kNL; ++l) n += kCi[l] * kCo[l] * kK[l] * kK[l] * kK[l] + kCo[l];
  return n;
}

// Host buffer in the reference layout: per layer w[co][ci][kz][ky][kx] then b[co].
int sgmg_unet_set_params(sgmg_unet* u, const float* host, void* stream) {
  if (!u || !host) { set_err("NULL argument"); return SGMG_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  size_t off = 0;
  for (int l = 0; l < kNL; ++l) {
    ULayer& L = u->L[l];
    std::vector<float> w(L.nw, 0.f);
    for (int co = 0; co < L.co; ++co)
      for (int ci = 0; ci < L.ci; ++ci)
        for (int t = 0; t < L.k3; ++t)
          w[((size_t)ci * L.k3 + t) * L.cop + co] = host[off + ((size_t)co * L.ci + ci) * L.k3 + t];
    off += (size_t)L.co * L.ci * L.k3;
    upload_layer(L, w, host + off, s);
    off += L.co;
    hipMemsetAsync(L.mw, 0, L.nw * sizeof(float), s);
    hipMemsetAsync(L.vw, 0, L.nw * sizeof(float), s);
    hipMemsetAsync(L.mb, 0, L.cop * sizeof(float), s);
    hipMemsetAsync(L.vb, 0, L.cop * sizeof(float), s);
  }
  u->step = 0;
  if (hipStreamSynchronize(s) != hipSuccess) { set_err("sync failed"); return SGMG_EHIP; }
  return check();
}

static int copy_out(sgmg_unet* u, float* host, bool grads, bool quantized, hipStream_t s) {
  size_t off = 0;
  for (int l = 0; l < kNL; ++l) {
    const ULayer& L = u->L[l];
    std::vector<float> w(L.nw), b(L.co);
    const float* srcw = grads ? L.gw : (quantized ? L.wq : L.w);
    const float* srcb = grads ? L.gb : L.b;
    hipMemcpyAsync(w.data(), srcw, L.nw * sizeof(float), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(b.data(), srcb, L.co * sizeof(float), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) { set_err("sync failed"); return SGMG_EHIP; }
    for (int co = 0; co < L.co; ++co)
      for (int ci = 0; ci < L.ci; ++ci)
        for (int t = 0; t < L.k3; ++t)
          host[off + ((size_t)co * L.ci + ci) * L.k3 + t] = w[((size_t)ci * L.k3 + t) * L.cop + co];
    off += (size_t)L.co * L.ci * L.k3;
    std::memcpy(host + off, b.data(), L.co * sizeof(float));
    off += L.co;
  }
  return 0;
}

int sgmg_unet_get_params(sgmg_unet* u, int quantized, float* host, void* stream) {
  if (!u || !host) { set_err("NULL argument"); return SGMG_EINVAL; }
  return copy_out(u, host, false, quantized != 0, (hipStream_t)stream);
}

int sgmg_unet_forward(sgmg_unet* u, int N, int D, int H, int W, const float* in, float* out,
                      void* stream) {
  if (!u || !in || !out) { set_err("NULL argument"); return SGMG_EINVAL; }
  int rc = check_dims(N, D, H, W);
  if (rc) return rc;
  if ((rc = ensure_act(u, N, D, H, W))) return rc;
  hipStream_t s = (hipStream_t)stream;
  forward(u, N, D, H, W, in, s);
  hipMemcpyAsync(out, u->y, (size_t)N * 3 * D * H * W * sizeof(float), hipMemcpyDeviceToDevice, s);
  return check();
}

// Forward + masked-MSE loss + backward; grads_host (may be NULL) receives the
// gradients in the reference layout; with lr > 0 an Adam step follows.
static int loss_and_grad(sgmg_unet* u, int N, int D, int H, int W, const float* in,
                         const float* target, const float* mask, float lr, float* loss,
                         float* grads_host, hipStream_t s) {
  int rc = check_dims(N, D, H, W);
  if (rc) return rc;
  if ((rc = ensure_act(u, N, D, H, W))) return rc;
  forward(u, N, D, H, W, in, s);
  RedWs ws{u->partials, nullptr};
  launch_mse(u->y, target, mask, N, 3, D * H * W, u->gy, ws, u->sums, s);
  backward(u, N, D, H, W, in, s);
  if ((rc = check())) return rc;
  if (grads_host && (rc = copy_out(u, grads_host, true, false, s))) return rc;
  if (lr > 0.f) {
    ++u->step;
    for (int l = 0; l < kNL; ++l) {
      ULayer& L = u->L[l];
      launch_adam(L.w, L.wq, L.gw, L.mw, L.vw, (long)L.nw, lr, 0.9f, 0.999f, 1e-8f, u->step, 1, s);
      launch_adam(L.b, nullptr, L.gb, L.mb, L.vb, L.co, lr, 0.9f, 0.999f, 1e-8f, u->step, 0, s);
    }
  }
  hipMemcpyAsync(u->h_sums, u->sums, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) { set_err("sync failed"); return SGMG_EHIP; }
  if (loss) *loss = (float)(u->h_sums[0] / u->h_sums[1]);
  return check();
}

int sgmg_unet_grad(sgmg_unet* u, int N, int D, int H, int W, const float* in, const float* target,
                   const float* mask, float* loss, float* grads_host, void* stream) {
  if (!u || !in || !target || !grads_host) { set_err("NULL argument"); return SGMG_EINVAL; }
  return loss_and_grad(u, N, D, H, W, in, target, mask, 0.f, loss, grads_host, (hipStream_t)stream);
}

int sgmg_unet_train_step(sgmg_unet* u, int N, int D, int H, int W, const float* in,
                         const float* target, const float* mask, float lr, float* loss,
                         void* stream) {
  if (!u || !in || !target || !(lr > 0.f)) { set_err("bad argument"); return SGMG_EINVAL; }
  return loss_and_grad(u, N, D, H, W, in, target, mask, lr, loss, nullptr, (hipStream_t)stream);
}

}  // extern "C"
