// Host-side launchers of the HIP kernels (one declaration per entry).
#pragma once
#include "common.hpp"

namespace sgmg {

// ---- fine level (kernels_fine.hip) -----------------------------------------
void launch_simp(const double* in, double* E64, float* E32, int nel, int is_modulus,
                 double E0, double Emin, double p, hipStream_t s);
void launch_mask_from_dofs(const uint8_t* fixed_dof, uint8_t* fixn, int Nn, hipStream_t s);
void launch_mask_cantilever(const Grid& g, uint8_t* fixn, hipStream_t s);
void launch_mask_inject(const Grid& fine, const Grid& coarse, const uint8_t* ffix,
                        uint8_t* cfix, hipStream_t s);
void launch_diag_fine(const Grid& g, const double* E, const double* ke, const uint8_t* fixn,
                      double* d, hipStream_t s);
template <typename T>
void launch_apply_fine_node(const Grid& g, const T* E, const T* ke, const T* u,
                            const uint8_t* fixn, const Epi<T>& ep, hipStream_t s);
// BF16 MFMA element kernel (kernels_mfma.hip); nsplit = 1 (BF16) or 3 (BF16X3);
// Launch shape (tuned per mesh): rows = element rows per wave tile (4 or 8),
// zchunk = owned node planes per wave.
void launch_apply_fine_mfma(const Grid& g, int nsplit, int rows, int zchunk, const float* Escaled,
                            const void* atab, const float* u, const uint8_t* fixn,
                            const Epi<float>& ep, hipStream_t s);
size_t apply_fine_mfma_blocks(const Grid& g, int rows, int zchunk);
bool mfma_shape_valid(int rows, int zchunk);
// The BF16-family MFMA kernel addresses vectors with 32-bit byte offsets
// below 2^30 (about 89 M nodes).
bool mfma_size_ok(const Grid& g);
// FP64 fine operator on the FP64 MFMA (same launch shapes).
void launch_apply_fine_mfma64(const Grid& g, int rows, int zchunk, const double* E,
                              const double* atab64, const double* u, const uint8_t* fixn,
                              const Epi<double>& ep, hipStream_t s);
bool mfma64_size_ok(const Grid& g);
void build_mfma_atab64(const KeTables& kt, double* out /* 2 * 6 * 64 */);
// FP64 fine operator on the vector ALU, element product in sum-factorised
// form (kernels_sf64.hip); zchunk = owned node planes per wave tile.
void launch_apply_fine_sf64(const Grid& g, int zchunk, const double* E, double lam, double mu,
                            const double* u, const uint8_t* fixn, const Epi<double>& ep,
                            hipStream_t s);
size_t apply_fine_sf64_blocks(const Grid& g, int zchunk);
bool sf64_size_ok(const Grid& g);
// Level-1 Galerkin product without the stored stencil (kernels_sf64.hip):
// E8 = the eight child moduli of each coarse element (zero where the element
// is not covered: a child with a Dirichlet DOF, or three children along an
// odd fine axis), skip = coarse nodes next to such an element (their rows
// come from the stencil, launch_stencil_apply_list).
void launch_l1_child_moduli(const Grid& fine, const Grid& coarse, const double* E,
                            const uint8_t* ffix, double* E8, uint8_t* el_out, hipStream_t s);
void launch_l1_skip_nodes(const Grid& coarse, const uint8_t* el_out, const uint8_t* cfix,
                          uint8_t* skip, hipStream_t s);
// One launch: the element products on the tiles and, in extra blocks, the
// listed rows (Sd, list) from their gathered stencil rows.
void launch_apply_l1_haar(const Grid& coarse, int zchunk, const double* E8, double lam, double mu,
                          const double* u, const uint8_t* fixn, const uint8_t* skip,
                          const double* Sd, const int* list, int nlist, const Epi<double>& ep,
                          hipStream_t s);
bool l1_haar_size_ok(const Grid& coarse);
void launch_scale_E(const double* E, float* Es, int nel, double inv_s, hipStream_t s);
void build_mfma_atab(const KeTables& kt, uint16_t* out /* 2 * 64 * 8 */);

// ---- stencil levels (kernels_stencil.hip) ----------------------------------
// Level-1 Galerkin aggregation: S1 = M1 sum_e E_e P_e^T (M_e K_e M_e) P_e M1.
// gtab: 27 pattern products G_p = P_p^T K_e P_p (24x24 each, pattern index
// px + 3 py + 9 pz), ke: K_e for the masked-child path.
void launch_galerkin_l1(const Grid& fine, const Grid& coarse, const double* E,
                        const double* gtab, const double* ke, const uint8_t* ffix,
                        const uint8_t* cfix, double* S, hipStream_t s);
void launch_galerkin_stencil(const Grid& fine, const Grid& coarse, const double* Sf,
                             const uint8_t* cfix, double* Sc, hipStream_t s);
void launch_stencil_diag(const Grid& g, const double* S, double* d, hipStream_t s);
void launch_stencil_to_f32(const double* S, float* S32, size_t n, hipStream_t s);
// form: 0 by node count, 1 LDS-staged 27-offset form, 2 plane-split form.
template <typename T>
void launch_stencil_apply(const Grid& g, const T* S, const T* u, const uint8_t* fixn,
                          const Epi<T>& ep, int form, hipStream_t s);
size_t stencil_apply_blocks(const Grid& g);
// The rows of the listed nodes gathered, once per assembly, into Sd
// (kStencil x nlist, entry-major) for launch_apply_l1_haar.
template <typename T>
void launch_stencil_gather_rows(const Grid& g, const T* S, const int* list, int nlist, T* Sd,
                                hipStream_t s);
// Restriction b_c = M_c P^T r_f; optionally x_c = c0 * Dinv_c * b_c (first
// smoothing step from zero) and d_c = x_c.
template <typename TF, typename TC>
void launch_restrict(const Grid& fine, const Grid& coarse, const TF* rf, const uint8_t* cfix,
                     TC* bc, const TC* dinv_c, double c0, TC* xc, TC* dc, hipStream_t s);
// Prolongation x_f += M_f P e_c.
template <typename TF, typename TC>
void launch_prolong_add(const Grid& fine, const Grid& coarse, const TC* ec, const uint8_t* ffix,
                        TF* xf, hipStream_t s);

// ---- vectors and reductions (kernels_vec.hip) ------------------------------
// out[k] = sum of partials[k * nblocks + b] over b (k < nv), one block.
void launch_finalize(RedWs ws, int nblocks, int nv, double* out, hipStream_t s);
void launch_power_start(double* x, const uint8_t* fixn, int Nn, uint64_t seed, hipStream_t s);
// out[0] = sum a*b (b == NULL: sum a*a; w != NULL: sum w*a*b)
int vec_dot_blocks(int n);   // block partials launch_dot writes for length n
void launch_dot(const double* a, const double* b, const double* w, int n, RedWs ws,
                double* out, hipStream_t s);
// y = Dinv * w ; out = ||y||^2
void launch_scale_dinv_norm(const double* dinv, const double* w, double* y, int n, RedWs ws,
                            double* out, hipStream_t s);
// x = y / sqrt(*nrm2)
void launch_normalize(const double* y, const double* nrm2, double* x, int n, hipStream_t s);
// V-cycle entry on level 0: b = (T) r ; d = c0 * Dinv * b ; x = d
template <typename T>
void launch_vcycle_entry(const double* r, T* b, const T* dinv, double c0, T* x, T* d, int n,
                         hipStream_t s);
void launch_d2f(const double* in, float* out, int n, hipStream_t s);
void launch_f2d(const float* in, double* out, int n, hipStream_t s);
void launch_copy(const double* in, double* out, int n, hipStream_t s);

// PCG pieces; sc = device scalar block (see runtime.hip for slots)
void launch_pcg_init(const double* f, const double* Ax0, int have_x0, double* r, int n,
                     RedWs ws, double* sc_ff_rr, hipStream_t s);
// x = x_in + alpha p (x_in may be x), r -= alpha q (alpha = sc[slot_rz] /
// p.q; a failed step leaves r and copies x_in to x), r.r; with b not NULL
// also the entry of the V-cycle that follows (b = (T) r, x = c0 Dinv b, d = x
// when d is not NULL).  p.q is sc[slot_pq], or, with pq_part not NULL, the
// sum of the npq block partials there (stored into sc[slot_pq]).  sc_rr
// NULL: the r.r partials stay in ws for launch_pcg_update_p_red.
template <typename T>
void launch_pcg_update_xr_entry(const double* x_in, double* x, double* r, double* r_old,
                                const double* p, const double* q, double* sc, int slot_rz,
                                int slot_pq, const double* pq_part, int npq, int n, RedWs ws,
                                double* sc_rr, T* b, const T* dinv, double c0, T* xe, T* de,
                                hipStream_t s);
// (sc_out2 NULL: partials only, for launch_pcg_update_p_red)
void launch_pcg_dot_rz(const double* r, const double* z, const double* r_old, int n, RedWs ws,
                       double* sc_out2, hipStream_t s);
// Block count (= partials per reduced value) of the vector kernels above.
int pcg_vec_partials(int n);
// p = z + beta p with the nrz r.z partials (then nrz r_old.z partials with
// flex) added in every block (no finalize launch); block 0 stores r.z [and
// r_old.z] at sc[slot_num] [slot_num + 1] and the sum of the r.r partials
// (pcg_vec_partials(n) of them) at sc[slot_rr]; with host not NULL (a
// device-mapped, coherent host array in sc's layout) it also writes those
// and sc[slot_pq] there, then increments the launch counter sc[slot_seq] and
// writes its new value to *host_seq (mapped too) after the scalars.
void launch_pcg_update_p_red(double* p, const double* z, const double* rz_part, int nrz,
                             const double* rr_part, double* sc, int slot_num, int flex,
                             int slot_den, int slot_rr, int slot_pq, int slot_seq, double* host,
                             double* host_seq, int n, hipStream_t s);
// *out = max over (free) entries of a non-negative vector (fixn may be NULL)
void launch_max_nonneg(const double* a, const uint8_t* fixn, int n, double* out, hipStream_t s);
void launch_diag_finalize(double* d, double* dinv64, float* dinv32, const uint8_t* fixn, int n,
                          const double* dmax, hipStream_t s);
void launch_apply_dinv(const double* dinv, const double* r, double* z, int n, hipStream_t s);
void launch_residual(const double* f, const double* Ax, double* r, int n, RedWs ws,
                     double* out_rr, hipStream_t s);

// ---- coarsest dense solve (kernels_dense.hip) ------------------------------
void launch_dense_assemble(const Grid& g, const double* S, const int* free_idx, int nf,
                           double* A, hipStream_t s);
void launch_dense_add_diag(double* A, int nf, const double* mean_diag_sum, hipStream_t s,
                           double* eps_out);
void launch_dense_diag_sum(const double* A, int nf, RedWs ws, double* out, hipStream_t s);
int dense_spd_inverse(double* A, int nf, double* scratch, int* d_flag, hipStream_t s);
// Symmetric coarsest solve from the packed upper-triangle tiles of Ainv:
// sym_tiles(nf) tiles of 64 x 64 doubles; partials 2 * sym_tiles(nf) * 64 doubles.
int sym_tiles(int nf);
void launch_dense_pack(const double* A, int nf, double* P, hipStream_t s);
void launch_dense_symv(const double* P, const int* free_idx, int nf, const double* r,
                       double* partials, double* z, hipStream_t s);

// Fixed-count Jacobi-PCG on the coarsest stencil from x = 0: 1 + 2 iters
// launches; r, z, the ping-pong pair p0/p1 and q each g.n doubles; scratch
// holds coarse_pcg_scratch(g, iters) doubles and done iters + 1 ints.
size_t coarse_pcg_scratch(const Grid& g, int iters);
void launch_coarse_pcg(const Grid& g, const double* S, const double* dinv, const uint8_t* fixn,
                       const double* b, double* x, double* r, double* z, double* p0, double* p1,
                       double* q, double* scratch, int* done, int iters, hipStream_t s);

// ---- flexible GMRES basis operations (kernels_krylov.hip) --------------------
void launch_basis_dots(const double* V, int ncols, const double* w, int n, RedWs ws, double* h_out,
                       hipStream_t s);
void launch_basis_update(double* w, const double* V, int ncols, const double* h, int n,
                         int next_dots, RedWs ws, double* out, hipStream_t s);
void launch_scale_inv_sqrt(const double* w, double* v, const double* nrm2, int n, hipStream_t s);
void launch_basis_combine(double* x, const double* Z, int k, const double* y, int n, hipStream_t s);
int basis_max_cols();

// ---- preconditioned Lanczos vector steps (kernels_krylov.hip) ----------------
void launch_lanczos_start(const double* g, const uint8_t* fixn, double* r, int n, hipStream_t s);
void launch_lanczos_resid(const double* sv, const double* w, const double* wp, double a, double b,
                          double* r, int n, hipStream_t s);
void launch_lanczos_next(const double* r, const double* z, double b, double* w, double* v, int n,
                         hipStream_t s);
size_t basis_partials(int ncols);

// ---- SIMP outer loop (kernels_simp.hip); element fields in x-fastest order --
void launch_filter_wsum(int nx, int ny, int nz, double rmin, double* W, hipStream_t s);
void launch_physical(int nx, int ny, int nz, double rmin, const double* W, const double* rho,
                     double beta, double eta, double* rhohat, double* dH, hipStream_t s);
void launch_element_energy(const Grid& g, const double* ke, const double* rhohat, const double* dH,
                           const double* u, double p, double E0, double Emin, double* gc,
                           RedWs ws, double* comp_out, hipStream_t s);
void launch_oc_ratio(int nx, int ny, int nz, double rmin, const double* W, const double* gc,
                     const double* dH, double* ratio, double* dc_out, double* dv_out,
                     hipStream_t s);
void launch_oc_volume(int nx, int ny, int nz, double rmin, const double* W, const double* rho,
                      const double* ratio, double lam, double move, double beta, double eta,
                      RedWs ws, double* vol_out, hipStream_t s);
int oc_apply_blocks(int n);
void launch_oc_apply(int n, double* rho, const double* ratio, double lam, double move, RedWs ws,
                     hipStream_t s);

}  // namespace sgmg
