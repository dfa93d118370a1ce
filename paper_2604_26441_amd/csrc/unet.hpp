// Launchers of the U-Net kernels (kernels_unet.hip).
#pragma once
#include "common.hpp"

struct sgmg_hierarchy;

namespace sgmg {

// A batch of samples on one mesh for the energy-norm training score.
struct EnergyBatch {
  Grid g;                  // fine node grid (all samples)
  const uint8_t* fixn;     // clamp bits per node
  const double* ke;        // K_e of the unit-modulus cube (576)
  const double* E;         // N x nel element moduli
  const double* f;         // N x ndof loads
  const double* cstar;     // N compliances f.u*
  double* u;               // N x ndof: network output as DOF vectors
  double* Ku;              // N x ndof
  double* part;            // N x nb x 2 block partials
  double* scal;            // N x 4: score, gradient factor, a / b, 0
  int N, nb;               // samples, node blocks of 256 per sample
  int Dp, Hp, Wp;          // padded voxel grid of the network
};
void launch_energy_loss(const EnergyBatch& e, const float* y, float* gy, hipStream_t s);

// Fine-level view of a hierarchy (runtime.hip) for the network's training.
struct FineView {
  Grid g;
  const uint8_t* fixn;
  const double* ke;
  int is_modulus;
  double E0, Emin, penal;
};
int hierarchy_fine_view(const ::sgmg_hierarchy* h, FineView* v);

void launch_conv_fwd(int K, const float* x, int N, int Ci, int Co, int D, int H, int W,
                     const float* w, const float* b, int relu, float* rpre, const float* add,
                     float* y, hipStream_t s);
size_t conv3_packed_words(int Ci, int Co);   // uint4 words of packed 3x3x3 weights
void launch_pack_conv3(const float* w, int Ci, int Co, uint4* wp, hipStream_t s);
// up = 1: x is stored at (D/2, H/2, W/2) and read as its nearest x2 upsampling
void launch_conv3_mfma(const float* x, int up, int N, int Ci, int Co, int D, int H, int W,
                       const uint4* wp, const float* b, int relu, float* rpre, const float* add,
                       float* y, hipStream_t s);
void launch_weight_transpose(const float* w, int Ci, int Co, int K, float* wt, hipStream_t s);
size_t conv_wgrad_part_floats(int N, int Ci, int Co, int D, int H, int W, int K);
void launch_conv_wgrad(int K, const float* x, int up, const float* dy, int N, int Ci, int Co, int D,
                       int H, int W, float* part, float* dw, float* db, hipStream_t s);
void launch_pool(const float* x, int NC, int D, int H, int W, float* y, hipStream_t s);
void launch_expand(const float* x, int NC, int D, int H, int W, float scale, float* y,
                   hipStream_t s);
void launch_sum8(const float* x, int NC, int D, int H, int W, float* y, hipStream_t s);
void launch_relu_bwd(const float* dy, const float* r, const float* extra, long n, float* dr,
                     hipStream_t s);
void launch_add(const float* a, const float* b, long n, float* y, hipStream_t s);
void launch_mse(const float* y, const float* t, const float* mask, int N, int C, int DHW, float* dy,
                RedWs ws, double* sums, hipStream_t s);
void launch_adam(float* p, float* pq, const float* g, float* m, float* v, long n, float lr, float b1,
                 float b2, float eps, int step, int quantize, hipStream_t s);
void launch_round_bf16(const float* p, float* q, long n, hipStream_t s);
void launch_unet_input(const Grid& g, const double* rho, const double* f, const uint8_t* fixn,
                       double* fmax_scratch, int Dp, int Hp, int Wp, float* in, hipStream_t s);
void launch_unet_output(const Grid& g, const float* out, const uint8_t* fixn, int Dp, int Hp,
                        int Wp, double* u, hipStream_t s);
void launch_unet_target(const Grid& g, const double* u, double* umax_scratch, int Dp, int Hp, int Wp,
                        float* t, float* m, hipStream_t s);
void launch_scale_by_ratio(double* u, int n, const double* num, const double* den, double* alpha,
                           hipStream_t s);

}  // namespace sgmg
