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
  uint4 *wp = nullptr, *wpt = nullptr;   // packed matrix-core operands (3x3x3 layers)
};

}  // namespace

struct sgmg_unet {
  ULayer L[kNL];
  std::vector<void*> mem;
  int step = 0;
  bool packed = false;        // wp holds the current BF16 weights
  // activation workspace for one (N, D, H, W)
  int aN = 0, aD = 0, aH = 0, aW = 0;
  std::vector<void*> act;
  float *r1 = nullptr, *p1, *r2, *p2, *r3, *p3, *r4, *r5, *d3, *r6, *d2, *r7, *d1,
        *y, *gy, *g1, *g2, *g3, *g4, *g5, *part;
  double* sums = nullptr;
  double* partials = nullptr;
  double h_sums[2];
  // energy-score workspace for eN samples of a mesh with eNn nodes
  int eN = 0, eNn = 0, enel = 0;
  std::vector<void*> emem;
  double *eE = nullptr, *eu, *eKu, *epart, *escal;
  float* eE32 = nullptr;
  std::vector<double> h_escal;
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

void free_energy(sgmg_unet* u) {
  for (void* p : u->emem) hipFree(p);
  u->emem.clear();
  u->eN = 0;
}

int ensure_energy(sgmg_unet* u, int N, const Grid& g) {
  if (u->eN == N && u->eNn == g.Nn && u->enel == g.nel) return 0;
  free_energy(u);
  const size_t nd = (size_t)N * g.n, nb = div_up(g.Nn, 256);
  struct Req { void** p; size_t bytes; };
  const Req reqs[] = {{(void**)&u->eE, (size_t)N * g.nel * 8}, {(void**)&u->eE32, (size_t)N * g.nel * 4},
                      {(void**)&u->eu, nd * 8}, {(void**)&u->eKu, nd * 8},
                      {(void**)&u->epart, N * nb * 2 * 8}, {(void**)&u->escal, (size_t)N * 4 * 8}};
  for (const Req& r : reqs) {
    void* v = nullptr;
    if (hipMalloc(&v, std::max<size_t>(r.bytes, 8)) != hipSuccess) {
      free_energy(u);
      set_err("U-Net energy workspace allocation failed");
      return SGMG_ENOMEM;
    }
    u->emem.push_back(v);
    *r.p = v;
  }
  u->h_escal.assign((size_t)N * 4, 0.0);
  u->eN = N; u->eNn = g.Nn; u->enel = g.nel;
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
      {&u->r3, N * 64 * v3}, {&u->p3, N * 64 * v4}, {&u->r4, N * 128 * v4},
      {&u->r5, N * 64 * v3}, {&u->d3, N * 64 * v3}, {&u->r6, N * 32 * v2},
      {&u->d2, N * 32 * v2}, {&u->r7, N * 16 * v1}, {&u->d1, N * 16 * v1},
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

// the 3x3x3 layers run on the matrix cores with packed weights, repacked
// after every change of the BF16 weights
void pack_weights(sgmg_unet* u, hipStream_t s) {
  if (u->packed) return;
  for (int l = 0; l < kNL; ++l)
    if (u->L[l].k == 3) launch_pack_conv3(u->L[l].wq, u->L[l].ci, u->L[l].co, u->L[l].wp, s);
  u->packed = true;
}

// up = 1: x holds the layer's input at half resolution and the convolution
// reads its nearest-neighbour upsampling (3x3x3 layers only)
void conv(sgmg_unet* u, int l, const float* x, int up, int N, int D, int H, int W, int relu,
          float* rpre, const float* add, float* y, hipStream_t s) {
  const ULayer& L = u->L[l];
  if (L.k == 3)
    launch_conv3_mfma(x, up, N, L.ci, L.co, D, H, W, L.wp, L.b, relu, rpre, add, y, s);
  else
    launch_conv_fwd(L.k, x, N, L.ci, L.co, D, H, W, L.wq, L.b, relu, rpre, add, y, s);
}

void forward(sgmg_unet* u, int N, int D, int H, int W, const float* x, hipStream_t s) {
  const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4, D4 = D / 8,
            H4 = H / 8, W4 = W / 8;
  pack_weights(u, s);
  conv(u, 0, x, 0, N, D, H, W, 1, nullptr, nullptr, u->r1, s);
  launch_pool(u->r1, N * 16, D, H, W, u->p1, s);
  conv(u, 1, u->p1, 0, N, D2, H2, W2, 1, nullptr, nullptr, u->r2, s);
  launch_pool(u->r2, N * 32, D2, H2, W2, u->p2, s);
  conv(u, 2, u->p2, 0, N, D3, H3, W3, 1, nullptr, nullptr, u->r3, s);
  launch_pool(u->r3, N * 64, D3, H3, W3, u->p3, s);
  conv(u, 3, u->p3, 0, N, D4, H4, W4, 1, nullptr, nullptr, u->r4, s);
  // the decoder convolutions read the upsampled tensors (up b, up d3, up d2)
  // through their input staging; those are never stored
  conv(u, 4, u->r4, 1, N, D3, H3, W3, 1, u->r5, u->r3, u->d3, s);
  conv(u, 5, u->d3, 1, N, D2, H2, W2, 1, u->r6, u->r2, u->d2, s);
  conv(u, 6, u->d2, 1, N, D, H, W, 1, u->r7, u->r1, u->d1, s);
  conv(u, 7, u->d1, 0, N, D, H, W, 0, nullptr, nullptr, u->y, s);
}

// dx = data gradient of layer l: the convolution with the channels swapped
// and the taps flipped
void conv_dgrad(sgmg_unet* u, int l, const float* dy, int N, int D, int H, int W, float* dx,
                hipStream_t s) {
  const ULayer& L = u->L[l];
  launch_weight_transpose(L.wq, L.ci, L.co, L.k, L.wt, s);
  if (L.k == 3) {
    launch_pack_conv3(L.wt, L.co, L.ci, L.wpt, s);
    launch_conv3_mfma(dy, 0, N, L.co, L.ci, D, H, W, L.wpt, nullptr, 0, nullptr, nullptr, dx, s);
  } else {
    launch_conv_fwd(L.k, dy, N, L.co, L.ci, D, H, W, L.wt, nullptr, 0, nullptr, nullptr, dx, s);
  }
}

void backward(sgmg_unet* u, int N, int D, int H, int W, const float* x, hipStream_t s) {
  const ULayer* L = u->L;
  const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4, D4 = D / 8,
            H4 = H / 8, W4 = W / 8;
  const long v1 = (long)D * H * W, v2 = v1 / 8, v3 = v2 / 8, v4 = v3 / 8;
  float *gd1 = u->g1, *gt = u->g2, *gd2 = u->g3, *gd3 = u->g4, *gt2 = u->g5;
  // output 1x1 conv
  launch_conv_wgrad(1, u->d1, 0, u->gy, N, 16, 3, D, H, W, u->part, L[7].gw, L[7].gb, s);
  conv_dgrad(u, 7, u->gy, N, D, H, W, gd1, s);                       // dL/d d1 (skip to e1 too)
  launch_relu_bwd(gd1, u->r7, nullptr, N * 16 * v1, gt, s);          // dL/d r7 pre
  launch_conv_wgrad(3, u->d2, 1, gt, N, 32, 16, D, H, W, u->part, L[6].gw, L[6].gb, s);
  conv_dgrad(u, 6, gt, N, D, H, W, gt2, s);                          // dL/d u2 [N,32,D]
  launch_sum8(gt2, N * 32, D, H, W, gd2, s);                         // dL/d d2 [N,32,D2]
  launch_relu_bwd(gd2, u->r6, nullptr, N * 32 * v2, gt, s);
  launch_conv_wgrad(3, u->d3, 1, gt, N, 64, 32, D2, H2, W2, u->part, L[5].gw, L[5].gb, s);
  conv_dgrad(u, 5, gt, N, D2, H2, W2, gt2, s);                       // dL/d u3 [N,64,D2]
  launch_sum8(gt2, N * 64, D2, H2, W2, gd3, s);                      // dL/d d3 [N,64,D3]
  launch_relu_bwd(gd3, u->r5, nullptr, N * 64 * v3, gt, s);
  launch_conv_wgrad(3, u->r4, 1, gt, N, 128, 64, D3, H3, W3, u->part, L[4].gw, L[4].gb, s);
  conv_dgrad(u, 4, gt, N, D3, H3, W3, gt2, s);                       // dL/d u4 [N,128,D3]
  launch_sum8(gt2, N * 128, D3, H3, W3, gt, s);                      // dL/d r4 [N,128,D4]
  launch_relu_bwd(gt, u->r4, nullptr, N * 128 * v4, gt2, s);
  launch_conv_wgrad(3, u->p3, 0, gt2, N, 64, 128, D4, H4, W4, u->part, L[3].gw, L[3].gb, s);
  conv_dgrad(u, 3, gt2, N, D4, H4, W4, gt, s);                       // dL/d p3 [N,64,D4]
  launch_expand(gt, N * 64, D3, H3, W3, 0.125f, gt2, s);             // pool adjoint
  launch_relu_bwd(gt2, u->r3, gd3, N * 64 * v3, gt, s);              // + skip from d3
  launch_conv_wgrad(3, u->p2, 0, gt, N, 32, 64, D3, H3, W3, u->part, L[2].gw, L[2].gb, s);
  conv_dgrad(u, 2, gt, N, D3, H3, W3, gt2, s);                       // dL/d p2 [N,32,D3]
  launch_expand(gt2, N * 32, D2, H2, W2, 0.125f, gt, s);
  launch_relu_bwd(gt, u->r2, gd2, N * 32 * v2, gt2, s);              // + skip from d2
  launch_conv_wgrad(3, u->p1, 0, gt2, N, 16, 32, D2, H2, W2, u->part, L[1].gw, L[1].gb, s);
  conv_dgrad(u, 1, gt2, N, D2, H2, W2, gt, s);                       // dL/d p1 [N,16,D2]
  launch_expand(gt, N * 16, D, H, W, 0.125f, gt2, s);
  launch_relu_bwd(gt2, u->r1, gd1, N * 16 * v1, gt, s);              // + skip from d1
  launch_conv_wgrad(3, x, 0, gt, N, 5, 16, D, H, W, u->part, L[0].gw, L[0].gb, s);
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
  free_energy(u);
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
    if (!rc && L.k == 3) {
      float* a = nullptr;
      rc = ualloc(u->mem, &a, 4 * conv3_packed_words(L.ci, L.co));
      L.wp = (uint4*)a;
      if (!rc) rc = ualloc(u->mem, &a, 4 * conv3_packed_words(L.co, L.ci));
      L.wpt = (uint4*)a;
    }
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
  u->packed = false;
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

// Backward from the output gradient u->gy; grads_host (may be NULL) receives
// the gradients in the reference layout; with lr > 0 an Adam step follows.
static int backward_and_step(sgmg_unet* u, int N, int D, int H, int W, const float* in, float lr,
                             float* grads_host, hipStream_t s) {
  int rc;
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
    u->packed = false;
  }
  return 0;
}

// Forward + masked-MSE loss + backward (+ Adam with lr > 0).
static int loss_and_grad(sgmg_unet* u, int N, int D, int H, int W, const float* in,
                         const float* target, const float* mask, float lr, float* loss,
                         float* grads_host, hipStream_t s) {
  int rc = check_dims(N, D, H, W);
  if (rc) return rc;
  if ((rc = ensure_act(u, N, D, H, W))) return rc;
  forward(u, N, D, H, W, in, s);
  RedWs ws{u->partials, nullptr};
  launch_mse(u->y, target, mask, N, 3, D * H * W, u->gy, ws, u->sums, s);
  if ((rc = backward_and_step(u, N, D, H, W, in, lr, grads_host, s))) return rc;
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

int sgmg_unet_energy_step(sgmg_unet* u, const sgmg_hierarchy* h, int N, int D, int H, int W,
                          const float* in, const double* rho_or_E, const double* f,
                          const double* cstar, float lr, float* loss, float* grads_host,
                          void* stream) {
  if (!u || !h || !in || !rho_or_E || !f || !cstar || !(lr >= 0.f)) {
    set_err("bad argument");
    return SGMG_EINVAL;
  }
  FineView fv;
  int rc = hierarchy_fine_view(h, &fv);
  if (rc) return rc;
  if ((rc = check_dims(N, D, H, W))) return rc;
  if (D < fv.g.Nz || H < fv.g.Ny || W < fv.g.Nx) {
    set_err("padded volume smaller than the node grid");
    return SGMG_EINVAL;
  }
  if ((rc = ensure_act(u, N, D, H, W)) || (rc = ensure_energy(u, N, fv.g))) return rc;
  hipStream_t s = (hipStream_t)stream;
  forward(u, N, D, H, W, in, s);
  launch_simp(rho_or_E, u->eE, u->eE32, N * fv.g.nel, fv.is_modulus, fv.E0, fv.Emin, fv.penal, s);
  EnergyBatch e;
  e.g = fv.g; e.fixn = fv.fixn; e.ke = fv.ke; e.E = u->eE; e.f = f; e.cstar = cstar;
  e.u = u->eu; e.Ku = u->eKu; e.part = u->epart; e.scal = u->escal;
  e.N = N; e.nb = (int)div_up(fv.g.Nn, 256); e.Dp = D; e.Hp = H; e.Wp = W;
  launch_energy_loss(e, u->y, u->gy, s);
  if ((rc = backward_and_step(u, N, D, H, W, in, lr, grads_host, s))) return rc;
  hipMemcpyAsync(u->h_escal.data(), u->escal, (size_t)N * 4 * sizeof(double),
                 hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) { set_err("sync failed"); return SGMG_EHIP; }
  double tot = 0.0;
  for (int n = 0; n < N; ++n) tot += u->h_escal[4 * (size_t)n];
  if (loss) *loss = (float)(tot / N);
  return check();
}

}  // extern "C"
