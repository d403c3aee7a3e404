// Host-callable launchers of the HIP kernels (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mlmc {

// rng.hip
hipError_t launch_draw_xi(uint64_t seed, int level, uint64_t first, int64_t count, int M,
                          double* xi, hipStream_t st, int stream = 0);
// row r: sample ids[r] of level lv[r] into row slots[r] of xi
// b = (h^3 / 8) sum of the 8 element values of f around each interior node of
// mesh n (grid layout, boundary positions 0), B samples
hipError_t launch_load(int n, int B, const double* f, double* b, hipStream_t st);
// The whole mixed-precision solve of B samples on an n^3 mesh (n = 4 or 8),
// one workgroup per sample: fp64 refinement (u, r = b - A u with the fp64
// kappa) around fp32 GMG-PCG to inner_rtol with the V-cycle of launch_vsmall
// (Chebyshev degree/coefficients c1, c2); b = bvec (grid layout) or bconst at
// every interior node.  Writes u (grid layout), active (0 where converged to
// rtol) and iters (inner iterations); rr_out (may be null) the last fp64
// ||b - A u||^2.  A NaN or Inf residual ends a sample's solve (active 0, rr_out
// non-finite).
hipError_t launch_solve_small(int n, int B, int degree, const double* c1, const double* c2, const double* kap,
                              const double* bvec, double bconst, double* u, int* active, int* iters, double rtol,
                              double inner_rtol, int max_iter, int max_outer, hipStream_t st,
                              double* rr_out = nullptr);
hipError_t launch_pause_draw(uint64_t seed, int level, int64_t count, double a, double w, double* out,
                             hipStream_t st);
// every workgroup w < nwg waits spin[w] ticks of the device wall clock and adds
// the ticks it measured to meas[w]
hipError_t launch_pause_spin(const uint32_t* spin, uint64_t* meas, int nwg, hipStream_t st);
hipError_t launch_draw_xi_rows(uint64_t seed, int64_t count, int M, const uint64_t* ids, const int* lv,
                               const int* slots, double* xi, hipStream_t st);

// field.hip: kappa[b][e] = exp(sum_m xi[b][m] sqrtlam[m] tab[ex][t0] tab[ey][t1] tab[ez][t2])
// rowmap (may be null): row r reads xi row rowmap[r] and writes kappa slot rowmap[r]
// bf16: the contraction with bf16 operands and fp32 accumulation
// xperm/xoff (not bf16): the separable evaluation (modes grouped by x-factor)
// instead of the dense MFMA GEMM
hipError_t launch_field(int n, int M, int64_t count, const double* xi, const double* sqrtlam,
                        const int* triples, const double* tab, int K1, double* kappa,
                        float* kappa32, hipStream_t st, const int* rowmap = nullptr, bool bf16 = false,
                        const int* xperm = nullptr, const int* xoff = nullptr);

// Per-sample scalar state of a batched Krylov solve (device arrays of B entries).
struct SolveState {
  double* rz;       // r . z of the current iteration
  double* alpha;
  double* beta;
  double* rr;       // ||r||^2
  double* bb;       // ||b||^2
  double* partial;  // [B][pstride] partial sums of the current reduction
  int* active;      // 1 while the sample iterates
  int* iters;       // iterations done
  int* nactive;     // single counter (device) of active samples
  uint32_t pstride; // capacity of partial sums per sample
  int* phase;       // serving: per-slot phase (PHASE_*), may be null
  int* pstate;      // fused-direction PCG: bit 0 = buffer of the current direction, bit 1 = no step taken yet,
                    // bit 2 = the iterate holds no value yet (written, not updated, by its first update),
                    // bit 3 = buffer of the current residual (fused residual update)
  int* began;       // fused-direction PCG: samples active when the solve started
};

// per-slot phases of a served batch
enum : int { PHASE_FREE = 0, PHASE_INNER = 1, PHASE_TRANSITION = 2, PHASE_RESTART = 3, PHASE_DONE = 4 };

// Grid-layout kernels on an n^3 mesh for `B` samples; `active` (may be null)
// skips samples whose flag is 0.  Device pointers must be 16-byte aligned.
// z-march variants (bit flags), chosen per context by measurement
// stencil engine variant bits: register window (0), register window with the
// next plane prefetched (ZVAR_PREFETCH), LDS-tiled planes for the plain kernels
// (ZVAR_LDS) and for the step that applies the coarse-grid correction
// (ZVAR_LDS_PRO)
enum : int { ZVAR_PREFETCH = 1, ZVAR_LDS = 2, ZVAR_LDS_PRO = 4 };

template <class T>
hipError_t launch_apply(int n, int B, const T* kap, const T* u, T* y, const int* active, hipStream_t st,
                        int var = 0);
template <class T>
hipError_t launch_residual(int n, int B, const T* kap, const T* b, const T* x, T* r,
                           const int* active, hipStream_t st, int var = 0);
// Chebyshev step.  zero_x: out = c2 D^-1 b (x0 = 0).  Otherwise
// out = x + c1 (x - xo) + c2 D^-1 (b - A x), where use_xo == 0 takes xo = 0.
// out may alias xo, never x.  With `dot` (non-zero-x steps on meshes n >= 4)
// the kernel also writes partial sums of b . out into dot->partial.
template <class T>
hipError_t launch_cheb(int n, int B, const T* kap, const T* b, const T* x, const T* xo, T* out,
                       double c1, double c2, bool zero_x, bool use_xo, const int* active,
                       hipStream_t st, SolveState* dot = nullptr, uint32_t* nparts = nullptr,
                       int var = 0);
// First post-smoothing step fused with the coarse-grid correction:
// out = y + c2 D^-1 (b - A y) with y = x + P xc (xc on the n/2 mesh, P the
// trilinear prolongation), n >= 4.  save (may be null) receives y.  out and
// save must not alias x, xc or each other.  `dot` as in launch_cheb.
template <class T>
hipError_t launch_cheb_prolong(int n, int B, const T* kap, const T* b, const T* x, const T* xc, T* out, T* save,
                               double c2, const int* active, hipStream_t st, SolveState* dot = nullptr,
                               uint32_t* nparts = nullptr, int var = 0);
// x += alpha p, r -= alpha q (alpha = s.alpha[b]), partial sums of r . r into
// s.partial, and z = c2 D^-1 r: a PCG update fused with the zero-iterate
// Chebyshev step of the following V-cycle (n >= 4).
template <class T>
hipError_t launch_pcg_update_zero(int n, int B, const T* kap, T* x, const T* p, T* r, const T* q, T* z, double c2,
                                  SolveState s, uint32_t* nparts, hipStream_t st, int var = 0);
template <class T>
hipError_t launch_restrict(int nf, int B, const T* rf, T* bc, const int* active, hipStream_t st);
// bc = P^T (b - A x) on the n/2 mesh (full weighting of the residual, which is
// never stored); usable when resr_usable(n, B) (LDS-tiled, n >= 4)
template <class T>
bool resr_usable(int n, int B);
// presmooth: the operand x is not read but formed on the fly as c2 D^-1 b (the
// zero-start Chebyshev step of a V-cycle level), i.e. bc = P^T (b - A c2 D^-1 b);
// usable when presmooth_usable(n, B)
template <class T>
hipError_t launch_residual_restrict(int n, int B, const T* kap, const T* b, const T* x, T* bc, const int* active,
                                   hipStream_t st, bool presmooth = false, double c2 = 0.0);
template <class T>
bool presmooth_usable(int n, int B);
// launch_cheb_prolong with the pre-smoothed iterate formed on the fly:
// out = y + c2 D^-1 (b - A y), y = c2 D^-1 b + P xc (one Chebyshev step on each
// side of the coarse-grid correction, the first from a zero iterate)
// b1/bstate (may be null): the right-hand side of sample s is b1 where
// (bstate[s] & 8) (the second residual buffer of a fused-update PCG)
template <class T>
hipError_t launch_cheb_prolong_presmoothed(int n, int B, const T* kap, const T* b, const T* xc, T* out, double c2,
                                           const int* active, hipStream_t st, SolveState* dot = nullptr,
                                           uint32_t* nparts = nullptr, const T* b1 = nullptr,
                                           const int* bstate = nullptr);
// The pre-smoothed residual restriction with the PCG residual update of the
// previous iteration fused in: r = r_old - alpha q (r_old in r0 or r1 by
// s.pstate bit 3; not on a first iteration, s.pstate bit 1) formed on the fly,
// written to the other buffer, partial sums of r . r into s.partial (*nparts
// per sample); bc = P^T (r - A c2 D^-1 r).  Usable when presmooth_usable.
template <class T>
hipError_t launch_residual_restrict_update(int n, int B, const T* kap, const T* r0, T* r1, const T* q, T* bc,
                                          SolveState s, double c2, uint32_t* nparts, hipStream_t st);
template <class T>
hipError_t launch_prolong_add(int nf, int B, const T* xc, T* xf, const int* active, hipStream_t st);
template <class T>
hipError_t launch_coarsest(int B, const T* kap, const T* b, T* x, const int* active, hipStream_t st);
template <class T>
hipError_t launch_coarsen(int nf, int B, const T* kf, T* kc, hipStream_t st, const int* active = nullptr);
template <class Ts, class Td>
hipError_t launch_convert(size_t count, const Ts* src, Td* dst, hipStream_t st);
template <class T>
hipError_t launch_fill_interior(int n, int B, T* v, double value, const int* active, hipStream_t st);

// vsmall.hip -- the whole V-cycle from an n0^3 mesh (n0 <= 16) down to 2^3 in
// one kernel, one workgroup per sample, all coarse data in LDS.
// kap_levels[l] is the kappa of mesh n0 >> l; b, x are grid-layout n0 vectors.
template <class T>
size_t vsmall_lds_bytes(int n0);
template <class T>
hipError_t launch_vsmall(int n0, int B, int degree, const double* c1, const double* c2,
                         const T* const* kap_levels, const T* b, T* x, const int* active,
                         hipStream_t st);

// PCG building blocks, fp64 scalars and partial sums.  Launchers that write
// partial sums report in *nparts how many per sample they wrote.
template <class T>
hipError_t launch_pcg_apply_dot(int n, int B, const T* kap, const T* p, T* q, SolveState s,
                                uint32_t* nparts, hipStream_t st, int var = 0);
template <class T>
hipError_t launch_pcg_update(int n, int B, T* x, const T* p, T* r, const T* q, SolveState s,
                             uint32_t* nparts, hipStream_t st);
template <class T>
hipError_t launch_dot(int n, int B, const T* a, const T* b, SolveState s, uint32_t* nparts,
                      hipStream_t st);
// fused-direction PCG (direction buffers p0, p1 selected per sample by s.pstate):
// r -= alpha q with the partial sums of r . r
template <class T>
hipError_t launch_pcg_rupdate(int n, int B, T* r, const T* q, SolveState s, uint32_t* nparts, hipStream_t st);
// x += alpha p on samples with mask[b] that took a step (the update still owed)
template <class T>
hipError_t launch_pcg_finish(int n, int B, T* x, const T* p0, const T* p1, const int* mask, SolveState s,
                             hipStream_t st);
// began = active; pstate = first direction in buffer 0 on active samples (fresh:
// the iterate holds no value yet; it is written, not updated, by its first update)
hipError_t launch_dir_begin(int B, SolveState s, bool fresh, hipStream_t st);
// p = z + beta p_old formed while staging, written to the other buffer, q = A p,
// partial sums of p . q, and the previous x += alpha p_old (LDS engine, n >= 4,
// when dir_usable)
template <class T>
bool dir_usable(int n, int B);
template <class T>
hipError_t launch_pcg_dir_apply(int n, int B, const T* kap, const T* z, T* x, T* p0, T* p1, T* q, const int* pstate,
                                SolveState s, uint32_t* nparts, hipStream_t st);
// r -= alpha q, partial sums of r . r, z = c2 D^-1 r (no iterate update)
template <class T>
hipError_t launch_pcg_rupdate_zero(int n, int B, const T* kap, T* r, const T* q, T* z, double c2, SolveState s,
                                   uint32_t* nparts, hipStream_t st, int var = 0);
template <class T>
hipError_t launch_pcg_direction(int n, int B, const T* z, T* p, SolveState s, hipStream_t st);
// outer residual of the refinement loop: r = b - A x in fp64 plus ||r||^2 partials
// One fp64 refinement step with the inner correction applied on the fly:
// uout = u + d (u may be null: zero), rin = fp32(bconst - A uout), partial sums
// of (bconst - A uout) . itself in fp64.  uout must not alias u or d.
hipError_t launch_refine(int n, int B, const double* kap, double bconst, const double* u, const float* d,
                         double* uout, float* rin, SolveState s, uint32_t* nparts, hipStream_t st, int var = 0, const double* bvec = nullptr);
// launch_refine with the update the fused-direction inner solve still owes d
// applied on the fly: the correction is d + alpha p (alpha p for a fresh d),
// p the inner state's current direction (buffers p0/p1, inner.pstate,
// inner.alpha).  Usable when refine_owed_usable(n, B, var).
bool refine_owed_usable(int n, int B, int var);
hipError_t launch_refine_owed(int n, int B, const double* kap, double bconst, const double* u, const float* d,
                              const float* p0, const float* p1, SolveState inner, double* uout, float* rin,
                              SolveState s, uint32_t* nparts, hipStream_t st, const double* bvec = nullptr);
hipError_t launch_true_residual(int n, int B, const double* kap, double bconst, const double* x,
                                double* r, SolveState s, uint32_t* nparts, hipStream_t st,
                                int var = 0, const double* bvec = nullptr);
// p = z on active samples (vectorized copy of the planes 1..n-1 range)
template <class T>
hipError_t launch_copy(int n, int B, const T* z, T* p, SolveState s, hipStream_t st);
// x64 += d (fp32 correction) on active samples
hipError_t launch_add_correction(int n, int B, double* x, const float* d, SolveState s,
                                 hipStream_t st);
// r32 = (float) r64 on active samples
hipError_t launch_demote(int n, int B, const double* r, float* r32, SolveState s, hipStream_t st);

enum ReduceOp : int {
  RED_BB = 0,       // bb = sum
  RED_ALPHA = 1,    // alpha = rz / sum; iters += 1
  RED_RR = 2,       // rr = sum; converged when rr <= tol2 * bb -> active = 0
  RED_RZ_INIT = 3,  // rz = sum
  RED_BETA = 4,     // beta = sum / rz; rz = sum
  RED_STORE = 5,    // out[b] = sum (ignores the active mask)
  RED_RR_INNER = 6, // rr = sum; converged -> phase TRANSITION
  RED_RR_OUTER = 7, // rr = sum; phase DONE if converged else RESTART
  RED_BETA_DIR = 8, // fused direction: beta = sum / rz (not on a first direction); rz = sum
  RED_ALPHA_DIR = 9, // fused direction: alpha = rz / sum; iters += 1; next direction buffer, first cleared
  RED_RR_UPD = 10,   // fused residual update: as RED_RR, and the residual buffer flips unless first
  RED_RR_INNER_UPD = 11 // as RED_RR_INNER (serving), flip as RED_RR_UPD, and a converged slot leaves the mask
};
// The RR ops treat a NaN or Inf sum as the end of the sample's solve (active
// 0, or the DONE / TRANSITION phase), keeping the value in rr so the caller can
// tell it from convergence.
hipError_t launch_reduce(int B, int op, double tol2, uint32_t nparts, SolveState s, double* out,
                         hipStream_t st);

// Chan, Golub and LeVeque merge of the summary (nb, mb, m2b) into (n, mean, m2)
__host__ __device__ inline void chan_merge(double& n, double& mean, double& m2, double nb, double mb, double m2b) {
#pragma clang fp contract(off)
  if (nb == 0.0) return;
  const double nn = n + nb;
  const double d = mb - mean;
  mean = mean + d * (nb / nn);
  m2 = m2 + m2b + d * d * (n * nb / nn);
  n = nn;
}

// Level statistics fold (one workgroup per job): Y = qf - qc (qc may be null:
// Y = qf) for `count` samples in sample order, pushed into the record rec
// (layout: n, mean, m2, pn, pmean, pm2 as doubles, then the non-finite count
// as an unsigned 64-bit integer): complete blocks of kStatsBlock pushes are
// reduced by Welford in order and merged into (n, mean, m2) in block order;
// the pushes of an incomplete block stay in (pn, pmean, pm2).  Non-finite Y
// are counted, not pushed.
constexpr int kStatsBlock = 64;
constexpr int kMaxStatsJobs = 16;
struct StatsJob {
  const double* qf;
  const double* qc;
  uint64_t count;
  double* rec;
};
struct StatsJobs {
  StatsJob j[kMaxStatsJobs];
};
hipError_t launch_level_stats(int njobs, const StatsJobs& jobs, hipStream_t st);
hipError_t launch_count_active(int B, SolveState s, hipStream_t st);
// out[p] (one sample's grid stride) = interior unknown at position p, or -1
hipError_t launch_node_map(int n, int32_t* out, hipStream_t st);
// out[0] = number of b < B with mask[b] != 0 (one workgroup)
hipError_t launch_count_mask(const int* mask, int B, int* out, hipStream_t st);
hipError_t launch_set_active(int B, SolveState s, int value, hipStream_t st);

// partial sums of w . u into s.partial (reduce with RED_STORE)
hipError_t launch_qoi_partial(int n, int B, int qoi, const double* u, SolveState s,
                              uint32_t* nparts, hipStream_t st, bool masked = false);
hipError_t launch_phase_masks(int S, const int* phase, int* inner, int* trans, int* restart, int* done,
                              hipStream_t st);
hipError_t launch_set_phase_list(int count, const int* slots, int* phase, int value, hipStream_t st);
hipError_t launch_set_phase_mask(int S, const int* mask, int* phase, int value, int* zero, hipStream_t st);

// scratch.hip -- the static device scratch of the allocation-free entry point:
// its size, the lookup of the current device's copy (once per device, kept),
// and the QoI of B samples on mesh n with its partial sums there (rejects a
// batch whose partial sums exceed the scratch)
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch_init(int* device, void** out);
size_t qoi_scratch_bytes(int n, int B);
hipError_t launch_qoi_scratch(int n, int B, int qoi, const double* u, double* q, void* scratch_dev, hipStream_t st);

}  // namespace mlmc
