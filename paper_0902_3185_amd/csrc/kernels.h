// Kernel launchers shared by the host layer (api.cpp) and the .hip sources.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "macro.h"
#include "plan.h"

namespace dmrg {

constexpr int kPrecF64 = 0;
constexpr int kPrecF32 = 1;
constexpr int kPrecBF16X3 = 2;
constexpr int kMaxSegPerBlock = 32;

// y = alpha * H psi + beta * y with the fused kernel, from the tile images
// at images + slot * stride (words; see build_images): with wg_start null,
// nslots workgroups, workgroup b taking slot b; else nwg workgroups (a
// persistent launch), workgroup w taking slots wg_start[w] ..
// wg_start[w + 1] - 1 (a device array of nwg + 1 entries).  FP64: `dense` is the FP64 operator pool (A-side blocks
// k-major) and psi the FP64 vector.  FP32 and BF16X3: `dense` is the FP32
// pool (A-side blocks row-major, ndense elements) and psi32 an FP32 copy of
// psi (npsi elements); both buffers must hold at least 4 elements (vector
// loads are clamped inside them).  Events t0/t1, when not null, are recorded
// at the start and end of the kernel itself.
//
// Variants of the FP32 and BF16 products (the FP64 product has variant 0
// only): 0 = the 32 x 32 tile kernel above, sixteen waves per tile, one
// persistent workgroup per compute unit; 1 = the 64 x 64 macro-tile kernel
// (launch_hpsi_macro), for superblocks whose blocks are large.
constexpr int kVariants = 2;
hipError_t launch_hpsi(int prec, int variant, int nslots, const uint32_t* images, int32_t stride,
                       const void* dense, const double* psi, double* y, double alpha, double beta,
                       hipStream_t stream, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr,
                       const float* psi32 = nullptr, int64_t ndense = 0, int64_t npsi = 0,
                       const int32_t* wg_start = nullptr, int nwg = 0);

// out[0 .. n) = (float) psi, out[n .. n + kPoolPad) = 0
hipError_t launch_psi_to_f32(const double* psi, float* out, int64_t n, hipStream_t stream);

// y = alpha * H psi + beta * y with the macro-tile kernel (macro.h): nwg
// workgroups, workgroup w taking items wg_start[w] .. wg_start[w + 1] - 1,
// then a combining kernel over the nshared tiles listed in `shared` (tiles
// split between workgroups).  dense is the FP32 operator pool (ndense
// elements), psi32 the FP32 copy of psi (npsi elements), psi64 psi itself
// (elementwise terms are summed in FP64).  part holds the plan's nparts
// partial tiles (kMac * kMac floats each).  Both pools must be under 2 GiB.
// Events t0/t1 bracket the two kernels.
hipError_t launch_hpsi_macro(bool bf16, int nwg, int nshared, const MacTile* tiles, const MacSeg* segs,
                             const MacGG* ggs, const MacItem* items, const int32_t* wg_start,
                             const int32_t* shared, const float* dense, int64_t ndense, const float* psi32,
                             int64_t npsi, const double* psi64, double* y, double alpha, double beta,
                             float* part, hipStream_t stream, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// Writes c[refs[i].term] to the double at base + refs[i].off for i < n (the
// coefficient fields of staged tile images or segment tables), in stream
// order: products enqueued later see the new coefficients.  The coefficients
// travel as kernel arguments, kCoefBatch terms per launch.
constexpr int kCoefBatch = 240;
hipError_t launch_patch_coeffs(void* base, const CoefRef* refs, int64_t n, const double* c,
                               int32_t nterms, hipStream_t stream);

// The fixed device scratch of dmrg_hpsi_noalloc (noalloc.hip): kScratchFloats
// floats per device.  scratch_setup(device) looks up the device's copy once
// (hipGetSymbolAddress with that device current); scratch_ptr(device) returns
// it afterwards, or null if it was never set up.
constexpr int64_t kScratchFloats = (int64_t)1 << 24;   // 64 MiB
hipError_t scratch_setup(int device);
float* scratch_ptr(int device);

// partial[tile * stride + s] = < G tile, segment s of the tile with c = 1 >
hipError_t launch_term_dots(int prec, int ntiles, const TileDesc* tiles, const SegDesc* segs,
                            const void* dense, const int32_t* gsrc, const double* gscale,
                            const double* psi, const double* g, double* partial, int stride,
                            hipStream_t stream);

// The straightforward baseline: y *= beta, then one launch per (term, block).
hipError_t launch_plain(const std::vector<std::pair<SegDesc, TileDesc>>& work, int64_t D,
                        const double* dense, const int32_t* gsrc, const double* gscale,
                        const double* psi, double* y, double alpha, double beta,
                        hipStream_t stream);

// --- FP64 vector kernels for the Lanczos recursion (vec.hip) ---------------

// Number of partial sums the reductions below use for a vector of length n.
int vec_blocks(int64_t n);

// h[j] = < V_j, w >, j < nv (V_j = V + j*ldv); partial needs nv*vec_blocks(n).
hipError_t launch_multi_dot(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
                            double* partial, double* h, hipStream_t stream);

// w -= sum_j h[j] V_j, then nrm2[0] = ||w||^2 (partial: vec_blocks(n)).
hipError_t launch_multi_axpy_norm(double* w, const double* V, int64_t ldv, int nv,
                                  const double* h, int64_t n, double* partial, double* nrm2,
                                  hipStream_t stream);

// out = sum_j u[j] V_j  (u in device memory)
hipError_t launch_combine(double* out, const double* V, int64_t ldv, int nv, const double* u,
                          int64_t n, hipStream_t stream);

// dst = src * (1 / sqrt(*nrm2))   (the norm read on the device)
hipError_t launch_normalise(double* dst, const double* src, const double* nrm2, int64_t n,
                            hipStream_t stream);

// One step of the Lanczos recursion against the nv basis vectors
// V_0..V_{nv-1} (V_j = V_{nv-1} the current one), by classical Gram-Schmidt
// twice: h1 = V^T w; w -= V h1; h2 = V^T w; w -= V h2.  ab[0] = alpha_j =
// h1[j] + h2[j], ab[1] = beta_j = ||w||; vnext = w / beta_j (if vnext is not
// null).  partial needs lz_partial_size(n, nv) doubles.
size_t lz_partial_size(int64_t n, int nv);
// vnext32 (if not null, with vnext): an FP32 copy of vnext, for an FP32
// product of it (the same holds for out32 below).
hipError_t launch_lz_step(double* w, const double* V, int64_t ldv, int nv, int64_t n,
                          double* h1, double* h2, double* partial, double* ab, double* vnext,
                          hipStream_t stream, float* vnext32 = nullptr);

// A single-pass step (nv >= 2): the local three-term recurrence (alpha_j =
// <v_j, H v_j>, beta_{j-1}) followed by one Gram-Schmidt pass on the
// remainder, applied as one combined update whose coefficients come from one
// sweep for V^T w and V^T V_j; V_{j-1} must have left such a step (or a
// two-pass one) as its new vector.  It leaves its new vector
// unnormalised: out (if not null) receives x = H v_j - (recurrence and pass
// terms), nout its partial sums of ||x||^2 (lz_norm_partials(n) of them);
// the next step normalises it.  The current vector V_j is either stored
// normalised (npend null, beta_{j-1} = *beta_prev) or stored unnormalised
// by the previous step (npend = that step's nout): then w = H u for the
// stored u, the step normalises V_j in place and writes ab[-1] =
// beta_{j-1} = ||u||.  ab[0] = alpha_j, *scale = 1/||u|| (or 1), h the
// coefficients.  partial needs lz_partial_size(n, nv) doubles.  w is not
// modified.
size_t lz_norm_partials(int64_t n);
hipError_t launch_lz_step_onepass(double* w, double* V, int64_t ldv, int nv, int64_t n, double* h,
                                  double* partial, const double* npend, const double* beta_prev,
                                  double* nout, double* scale, double* ab, double* out,
                                  hipStream_t stream, float* out32 = nullptr);

// A recurrence-only step (nv >= 2, j = nv - 1): no pass over the basis.
// V_j is stored unnormalised by the previous step (npend = that step's
// nout) and w = H u for the stored u; the step normalises V_j in place and
// forms x = H v_j - alpha_j v_j - beta_{j-1} V_{j-1}, unnormalised, into out
// (if not null) with its partial sums of ||x||^2 in nout; ab[-1] =
// beta_{j-1} = ||u||, ab[0] = alpha_j = <v_j, H v_j>.  partial needs
// lz_norm_partials(n) doubles.  w is not modified.
hipError_t launch_lz_step_recurrence(const double* w, double* V, int64_t ldv, int nv, int64_t n,
                                     double* partial, const double* npend, double* nout,
                                     double* ab, double* out, hipStream_t stream,
                                     float* out32 = nullptr);

// Record alpha_j = h1[j] + h2[j] and beta_j = sqrt(nrm2) into ab[2*it], ab[2*it+1].
hipError_t launch_record(const double* h1, const double* h2, int j, const double* nrm2,
                         double* ab, int it, hipStream_t stream);

}  // namespace dmrg
