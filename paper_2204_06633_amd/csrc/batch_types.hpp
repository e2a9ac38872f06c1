// Descriptors and arguments of the batched kernels (shared by the kernels
// and the host layer).
#pragma once

#include <stdint.h>

#include "device_common.hpp"

namespace lr {

struct BatchTemplate {
  int64_t h_off;       // offset of h[0] in the batch h+ / hx arrays
  int64_t n_h;
  int64_t out_start;   // h-index of output sample 0
  int64_t n_out;
  int64_t out_off;     // offset of the output block (rows x n_out, channel-major)
  int64_t index;       // position in the caller's template list (sky row); < 0: empty slot
};

// Link samples of TDI halo that a fused work item of m templates and
// workgroups of `block` lanes carries from one tile to the next: the halo of
// every link row passes the next tile's projection in two registers per lane,
// and the rows are that much longer.  0 (no carrying) when fewer than 32
// samples would fit, at most 64.
constexpr int fused_halo_cap(int m, int block) {
  const int c = (2 * block / (6 * m)) & ~1;
  return c < 32 ? 0 : (c < 64 ? c : 64);
}

struct BatchFwdArgs {
  OrbitView orb_p, orb_t;
  const BatchTemplate* tpl;  // [n_groups * M], grouped, longest template first
  const int* items;          // [n_items][2]: group, segment
  int n_items;
  int* counter;              // work-item counter, zero before the launch
  double t_off_p, t_off_t;   // time of output sample 0 minus each orbit grid's first sample
  double dt, inv_dt;
  int F;                     // link samples before the first output of a tile
  int T_out;                 // outputs of a segment's first tile (even): link samples per
                             // tile minus the TDI halo
  int HP;                    // halo carried from tile to tile (link samples per tile -
                             // T_out), 0 for segments of one tile
  int seg_tiles;             // tiles per segment: T_out + (seg_tiles - 1) * link samples per
                             // tile outputs
  const double* hp;
  const double* hc;
  const double* sky;         // lam, beta of template k at sky[sky_stride * k + 0, 1]
  int sky_stride;            // 2 (sky array) or 8 (rows of params)
  const double* trig;        // [n_templates][4]: sin, cos of lam, then of beta (run_forward_prep)
  const double* params;      // [n_templates][8] or null: synthesise h+ / hx from these
  int channels;
  double* out;
};

struct BatchAdjTemplate {
  int64_t h_off, n_h;
  int64_t y_start, n_y;     // link series: h-indices [y_start, y_start + n_y)
  int64_t gy_off;           // offset of its [6][n_y] block in the link-gradient workspace
  int64_t out_off, n_out;
  int64_t index;            // caller's position (sky row, g_sky row, loglike entry)
  double t_off_h;           // time of h[0] minus the projection orbit grid's first sample
};

struct BatchAdjArgs {
  OrbitView orb_p, orb_t;
  const BatchAdjTemplate* tpl;  // [n_templates], caller's order
  const int64_t* items;         // [n_items][2]: template (TDI: pair), tile
  const int64_t* sky_items;     // [n][2]: template, tile of kBlock link samples (sky kernel)
  const int64_t* pairs;         // [n_pairs][2]: caller indices, longer first, -1 = none
  double t_off_y;               // time of link sample 0 (= output index -F) minus the TDI grid's
  double dt, inv_dt;
  int F;                        // link samples before output 0
  int channels;
  const double* hp;
  const double* hc;
  const double* sky;
  const double* g_out;
  double* g_y;
  double* g_hp;
  double* g_hc;
  double* sky_part;             // [n_sky_items][2] or null
  int rl_cap;                   // wave row capacity of the carry kernels (0: atomic kernels)
  int sky_stride;               // lam, beta of template k at sky[sky_stride * k + 0, 1]
  const double* params;         // [n][8] or null: waveform mode (see ProjAdjArgs)
  double* gb_part;              // waveform mode: [n_items][7] parameter-gradient sums
};

// Launchers (instantiated per tap count in batch_*.hip).
template <int N, int GEN, int M, int BLOCK, bool WAVE>
hipError_t launch_fused_forward(const BatchFwdArgs& a, int blocks, hipStream_t s);
template <int N, int GEN, int M, int BLOCK, bool WAVE>
int fused_occupancy();
template <int N, int GEN>
hipError_t launch_batch_tdi_adjoint(const BatchAdjArgs& a, int64_t n_items, hipStream_t s);
template <int N>
hipError_t launch_batch_project_adjoint(const BatchAdjArgs& a, int64_t n_items,
                                        int64_t n_sky_items, hipStream_t s);

// tile: link samples per work item (256, 512 or 1024; not 1024 with group
// 4); wave: waveform mode (h from a.params; groups 1, 2 at 512 and 2 at 1024)
hipError_t run_fused_forward(int order, int gen, int group, int tile, bool wave,
                             const BatchFwdArgs& a, int blocks, hipStream_t s);
int fused_blocks_per_cu(int order, int gen, int group, int tile, bool wave);
hipError_t run_batch_tdi_adjoint(int order, int gen, const BatchAdjArgs& a, int64_t n_items,
                                 hipStream_t s);
hipError_t run_batch_project_adjoint(int order, const BatchAdjArgs& a, int64_t n_items,
                                     int64_t n_sky_items, hipStream_t s);

}  // namespace lr
