// Host-side launchers of the ptymi kernels (one entry per kernel family).
#pragma once
#include <hip/hip_runtime.h>

#include "pty_common.hpp"

namespace pty {

// Prologue of the forward row pass: z = P S_j O, or z = 2 P S_j O - psi_j (DM).
enum class RowIn { Plain = 0, DmReflect = 1 };
// Per-pixel step of the column pass.  Poisson: the direction g Psi of the
// Poisson exit-wave update, g = 1 - d / (I + eps), with the two sums of its
// step length per (slot, column block) in poisp and the amplitude error.
enum class ColOp { Project = 0, NllGrad = 1, Intensity = 2, NllLoss = 3, Poisson = 4 };
// Epilogue of the inverse row pass.
enum class RowOut { DmUpdate = 0, StoreChi = 1, NllGrad = 2 };
// Object-tile gather: what is accumulated and how it is applied.
// Gradient writes the plain sum to `out`; WeightedSum writes the sum weighted
// by alpha[slot].x (LsqUpdate's numerator) to `out` without applying it.
enum class ObjOp { Density = 0, DmObject = 1, LsqDirection = 2, LsqUpdate = 3, Gradient = 4, WeightedSum = 5 };
// Probe reduction over positions.
enum class PrbOp { Plain = 0, AlphaWeighted = 1, Gradient = 2 };
// Probe apply step.
enum class PrbApply { Dm = 0, LsqDirection = 1, LsqUpdate = 2 };

struct FourierArgs {
  int n, k;
  const float2* obj;
  int h, w;
  const float2* probe;
  const int* jlist;       // pattern index of slot s = jlist[s]
  const PosInfo* pos;     // by pattern index
  const float* amp;       // J x N x N measured moduli (natural order), by pattern index
  float2* psi;            // DM exit waves J x K x N x N (by pattern index); may be null
  float2* chi;            // per-slot K x N x N (StoreChi / NllGrad); may be null
  float2* contrib;        // per-slot N x N sum_k conj(P_k) (.) ; may be null
  float2* zs;             // chunk scratch C x K x N x N
  double* errp;           // per (pattern index, column block) partials (2 doubles)
  double* posgrad;        // per (slot, row block) position-gradient partials (2 doubles)
  float* intensity_out;   // Intensity: J x N x N centred, by pattern index
  const float* tw;        // W_N table (N float2)
  int jl_off;             // chunk entry c reads pattern jlist[jl_off + c]
  int slot_off;           // ... and writes chi / contrib / posgrad slot slot_off + c
  int nc;                 // patterns in the chunk
  float nll_eps;
  float grad_scale;       // NllGrad: multiplies every gradient
  int masked;             // 1: the moduli carry a detector mask (sign bits)
  double* poisp;          // Poisson: per slot the step length alpha_R of the
                          // pattern (k_poisson_alpha); the StoreChi rows then
                          // scale by -alpha_R; null: the modulus projection's
                          // chi, unscaled
  float* pinten;          // Poisson: chunk x N x N model intensity (natural order)
  hipStream_t stream;
};

void launch_rows_fwd(const FourierArgs& a, RowIn mode);
void launch_cols(const FourierArgs& a, ColOp op);
void launch_rows_inv(const FourierArgs& a, RowOut mode);
// Poisson: the step length of every pattern of the chunk (one block each)
void launch_poisson_alpha(const FourierArgs& a);
int col_blocks(int n, int k);   // column blocks per pattern in the column pass
int row_blocks(int n);   // row blocks per pattern in the row passes

struct ObjGatherArgs {
  int n;
  int h, w;
  const TileEntry* tiles;
  int ntiles;
  const PatchRef* refs;
  const PosInfo* pos;
  const float2* src;      // per-slot N x N complex contributions
  const float* pint;      // N x N probe intensity (Density)
  const float2* alpha;    // per-slot step lengths (LsqUpdate uses .x)
  float2* obj;            // object (DmObject, LsqUpdate: in/out)
  float2* out;            // LsqDirection: direction plane; Gradient: gradient plane
  float* den;             // Density: output; others: input
  unsigned* den_max;      // Density: atomic max (float bits); others: input
  float gamma;            // delta = gamma * max(den)
  float beta;             // LsqUpdate relaxation
  hipStream_t stream;
};
void launch_obj_gather(const ObjGatherArgs& a, ObjOp op);

struct ProbeAccArgs {
  int n, k;
  const float2* obj;
  int h, w;
  const int* jlist;
  const PosInfo* pos;
  const float2* src;      // per-slot (or per-pattern for DM) K x N x N
  int src_by_pattern;     // 1: src indexed by pattern index j (DM psi); 0: by slot
  const float2* alpha;    // AlphaWeighted: weight alpha[slot].y
  int s0, count;          // slots [s0, s0 + count)
  int per_slice;
  float2* part_num;       // slices x K x N x N
  float* part_den;        // slices x N x N
  unsigned* zero;         // if set, zeroed by the first thread (the max that the finish takes next)
  hipStream_t stream;
};
int probe_slices(int count, int per_slice);
int lsq_row_blocks(int n);   // row blocks per window of the LSQML step sums
int probe_per_slice(int n, int count);
int probe_slices_max(int n, int count);
void launch_probe_acc(const ProbeAccArgs& a, PrbOp op);

struct ProbeFinishArgs {
  int n, k, slices;
  const float2* part_num;
  const float* part_den;   // may be null (Gradient)
  float2* num;             // K x N x N
  float* den;              // N x N (may be null)
  unsigned* den_max;       // atomic max of den (float bits), may be null
  hipStream_t stream;
};
void launch_probe_finish(const ProbeFinishArgs& a);

struct ProbeApplyArgs {
  int n, k;
  const float2* num;
  const float* den;
  const unsigned* den_max;
  float gamma, beta;
  float2* probe;           // Dm: in/out; LsqUpdate: in/out
  float2* dir;             // LsqDirection: output
  hipStream_t stream;
};
void launch_probe_apply(const ProbeApplyArgs& a, PrbApply op);

struct LsqStepArgs {
  int n, k;
  const float2* obj;
  const float2* dobj;
  int h, w;
  const float2* probe;
  const float2* dprobe;
  const float2* chi;
  const float2* contrib;
  const float* pint;       // N x N scratch: sum_k |P_k|^2
  const float2* pq;        // N x N scratch: sum_k conj(P_k) dP_k
  const float* dint;       // N x N scratch: sum_k |dP_k|^2
  const int* jlist;
  const PosInfo* pos;
  int count;
  int probe_on;
  double* part;            // count x row_blocks x (5, or 9 with shift)
  float2* alpha;           // per slot
  float2* alpha_by_j;      // per pattern index (reporting)
  float2* shift;           // per slot (dy, dx) of the position refinement, or nullptr
  float max_shift;         // clip of each shift component, px
  hipStream_t stream;
};
void launch_lsq_steps(const LsqStepArgs& a);
// Probe modes (and DM exit waves, if psi != nullptr: J sets of K modes)
// replaced by the orthogonal modes of the probe's Gram eigenbasis; gram: K x K
// double2 scratch, mix: K x K float2 scratch.  No-op for k == 1.
void launch_orthogonalise_modes(float2* probe, float2* psi, int n, int k, int j, double2* gram, float2* mix,
                                hipStream_t s);
// pos[jlist[b]] += shift[b] for b < count, kept in [0, lim]
void launch_pos_update(PosInfo* pos, const int* jlist, const float2* shift, int count, int lim_y, int lim_x,
                       hipStream_t s);

// Device positions (J x 2 float32 y, x) -> PosInfo, clamped into [0, lim].
void launch_pos_from_yx(const float* yx, int count, int lim_y, int lim_x, PosInfo* out, hipStream_t s);
// Tile lists of the slots [0, count) of jlist built on the device: one
// TileEntry per object tile (ceil(h / kTileH) x ceil(w / kTileW) of them, in
// row-major tile order; cnt holds as many ints), refs at most
// device_tile_refs_max(n, count) entries.
size_t device_tile_refs_max(int n, int count);
void launch_build_tiles(const PosInfo* pos, const int* jlist, int count, int n, int h, int w, int* cnt,
                        TileEntry* tiles, PatchRef* refs, hipStream_t s);
// p[i] = i for i < n
void launch_iota_i32(int* p, int n, hipStream_t s);

struct EpieArgs {
  int n, k;
  float2* obj;
  int h, w;
  const float2* probe;
  float2* probe_out;
  const float2* chi;
  PosInfo pos;
  float alpha, beta;
  int probe_on;
  unsigned* maxes;         // 2 zeroed slots of this position: max sum_k |P_k|^2, max |S_j O|^2 (float bits)
  float2* patch;           // N x N scratch: the pre-update patch S_j O
  hipStream_t stream;
};
void launch_epie_update(const EpieArgs& a);

// ePIE positions of 512 x 512 windows (1 or 2 modes), one 64-lane wavefront
// per line: per position three launches (rows with the step maxima, columns
// with the projection, inverse rows with the probe update and the object
// update).  probe_out receives the updated probe; it may be the probe itself
// only when probe updates are off (then nothing is written).  zs: K x N x N scratch; patch,
// contrib: N x N scratch; maxw: epie_wide_max_words() floats; errw:
// epie_wide_err_words() doubles.  The position's error partials go to errp
// (pattern j, bpp column slots: the sums in the first, zeros in the rest).
struct EpieWideArgs {
  int n, k;
  float2* obj;
  int h, w;
  const float2* probe;    // K x N x N
  float2* probe_out;      // K x N x N: the updated probe
  const float* amp;       // J x N x N measured moduli (natural order)
  PosInfo pos;
  int j;                  // pattern index
  float2* zs;
  float2* patch;
  float2* contrib;
  float* maxw;
  double* errw;
  double* errp;
  int bpp;
  const float* tw;        // W_N table (N float2)
  float alpha, beta;
  int probe_on;
  int masked;
  hipStream_t stream;
};
bool epie_wide_supported(int n, int k);
size_t epie_wide_max_words();
size_t epie_wide_err_words();
void launch_epie_wide(const EpieWideArgs& a);

// A whole ePIE iteration in one workgroup (small windows): for each position
// in `order`, the exit waves, both 2-D transforms, the projection with its
// error partials and both updates stay in LDS; positions run in sequence
// inside the kernel.  The probe alternates between probe0 and probe1 (after an
// odd number of positions the updated probe is in probe1).
struct EpieRunArgs {
  int n, k;
  float2* obj;
  int h, w;
  float2* probe0;
  float2* probe1;
  const float* amp;
  const PosInfo* pos;
  const int* order;
  int count;
  double* errp;
  int bpp;                // column blocks per pattern of the error partials
  const float* tw;
  float alpha, beta;
  int probe_on;
  hipStream_t stream;
};
bool epie_fused_supported(int n, int k);
void launch_epie_fused(const EpieRunArgs& a);

struct DmInitArgs {
  int n, k;
  const float2* obj;
  int h, w;
  const float2* probe;
  const PosInfo* pos;
  int j;
  float2* psi;
  float2* contrib;
  hipStream_t stream;
};
void launch_dm_init(const DmInitArgs& a);

// Small utilities
void launch_fill_u32(unsigned* p, size_t n, unsigned v, hipStream_t s);
void launch_amplitude(const float* counts, float* amp, double* totals, int n, int j, hipStream_t s);
// Marks pixels without a measurement (mask[q] == 0, natural order, shared by
// all patterns) by the sign bit of their stored modulus; nullptr clears it.
void launch_apply_mask(float* amp, const unsigned char* mask, int n, int j, hipStream_t s);
// totals[j] = sum_q amp[j][q]^2 (FP64, one block per pattern)
void launch_amp_totals(const float* amp, double* totals, int n, int j, hipStream_t s);
// pint = sum_k |P_k|^2; `zero`, if set, is zeroed too (the max the density gather takes next)
void launch_probe_intensity(const float2* probe, float* pint, int n, int k, hipStream_t s, unsigned* zero = nullptr);
// out[*slot] = E of the partials (slot NULL: out[0]); advance: then ++*slot (the
// device-side iteration counter, so that a captured iteration can be replayed).
void launch_err_reduce(const double* errp, int count, double* out, hipStream_t s, int* slot = nullptr,
                       bool advance = false);
void launch_posgrad_reduce(const double* part, int count, int nrb, float* out, const int* jlist, hipStream_t s);
void launch_scale_f32(float* p, size_t n, float s, hipStream_t st);
void launch_scale_c64(float2* p, size_t n, float s, hipStream_t st);
void launch_pattern_totals(const float* x, double* totals, int n, int j, hipStream_t s);

// Spatial decomposition of the object into strips (one per GPU in a
// multi-GPU run): halo messages of object-plane rows, probe-sum messages,
// the update applied from exchanged sums, and the error partials.
struct HaloPlanes {
  float* plane[2];        // plane base (row 0 of the local array), as 32-bit words
  int words_per_row[2];   // 0: plane unused
  int row0;               // first local row of the message
};
// Copies `rows` rows of each used plane (plane 0 first) into msg.
void launch_halo_pack(const HaloPlanes& p, int rows, float* msg, hipStream_t s);
// Adds msg into (add) or overwrites (copy) the same rows of the planes.
void launch_halo_unpack(const HaloPlanes& p, int rows, const float* msg, bool add, hipStream_t s);
// out = sum of `count` messages of `words` floats each, in message order.
void launch_sum_messages(const float* const* msgs, int count, size_t words, float* out, hipStream_t s);
// atomic max (float bits) of a non-negative plane into *out
void launch_plane_max(const float* x, size_t n, unsigned* out, hipStream_t s);
enum class ObjApply { Dm = 0, LsqDirection = 1, LsqUpdate = 2 };
// Per pixel, with d = den + gamma * max(den): Dm: obj = (num + delta obj) / d;
// LsqDirection: dir = num / d (0 where d = 0); LsqUpdate: obj += beta num / d.
void launch_obj_apply(const float2* num, const float* den, const unsigned* den_max, float gamma, float beta,
                      float2* obj, float2* dir, size_t n, ObjApply op, hipStream_t s);
// Copies the error partials of local patterns to their global pattern rows.
void launch_err_scatter(const double* local, const int* jmap, int count, int per_pattern, double* global,
                        hipStream_t s);

// Learned initialiser data path and evaluation helpers.
void launch_fill_c64(float2* p, size_t n, float2 v, hipStream_t s);
void launch_poisson(const float* lam, float* out, size_t n, uint64_t seed, hipStream_t s);
// Network input (128 x 128 windows): u = F(P0) / |F(P0)| and
// g = conj(P0) / (|P0|^2 + 0.01 max |P0|^2) from probe mode 0, then per window
// the central 64 x 64 of g F^-1(A u), upsampled 2x, as 128 x 128 x (Re, Im).
void launch_seed_planes(const float2* probe, float2* u, float2* g, hipStream_t s);
void launch_seed_input_counts(const float* counts, int nb, const float2* u, const float2* g, float* x, hipStream_t s);
void launch_seed_input_amp(const float* amp, const int* jsel, int nb, const float2* u, const float2* g, float* x,
                           hipStream_t s);
void launch_targets(const float2* obj, int w, const PosInfo* pos, int j, int n, float* out, hipStream_t s);
int seed_chain_grid();   // spacing of the chain's coarse sample grid (object pixels)
void launch_seed_chain(const float* patches, const int2* place, int j, float2* S, int hc, int wc, float2* phasor,
                       hipStream_t s);
void launch_seed_stitch(const float* patches, const int2* place, const float2* phasor, const int* bin_beg,
                        const int* bin_idx, int bins_w, int bins_h, float2* obj, int h, int w, hipStream_t s);
size_t nrmse_part_doubles();
void launch_nrmse(const float2* o, const float2* t, const unsigned char* mask, size_t n, double* part, double* out,
                  hipStream_t s, int* slot = nullptr, bool advance = false);
void launch_set_i32(int* p, int v, hipStream_t s);
void launch_roi_mask(const float* den, const unsigned* den_max, float frac, size_t n, unsigned char* mask,
                     hipStream_t s);

}  // namespace pty

// The network (defined with its kernels); the seeding entry point runs its
// forward pass on the context's stream.
struct pty_cnn;
namespace pty {
float* cnn_input_buffer(pty_cnn* c);
int cnn_max_batch(const pty_cnn* c);
int cnn_device(const pty_cnn* c);
const float* cnn_forward_batch(pty_cnn* c, const float* x, int nb, hipStream_t s);

}  // namespace pty
