// lbell_launch.h - host-side launchers of the HIP kernels (internal).
#pragma once
#include "lbell_dev.h"

namespace lbd {

struct LaunchCS {
    const BoxDesc* boxes;
    const BoxRT* rt;
    const int* tile_box;
    int ntiles;
    const void* fin;
    void* fout;
    KParams kp;
    bool walls;
    int variant;            // 0 generic tiles, 1 row-wave, 2 row-wave with non-temporal stores
    bool aa;                // generic tiles in place on fin (== fout); kp.conv says even or odd step
    int spt;                // generic tiles: 256-site tiles per block (1 or 2)
    int xcd;                // generic tiles: block order, 0 plain, 1 XCD-chunked, 2 XCD-grouped
    bool nt;                // generic tiles: non-temporal stores
    int grid;               // generic tiles: blocks launched (0 = one per block of tiles; fewer = persistent)
    int rows_k;             // sites per lane of the row-wave kernel (nx = 64 rows_k), 0 = not applicable
    int rows_ny, rows_nz;   // its box (single-box contexts only)
    int part;               // 0 every block, 1 blocks not in the near set, 2 blocks of the near set
    const uint32_t* near_flags;
    const int* near_list;
    const int* near_count;
    uint32_t near_epoch;    // a block is near iff its flag equals this step's epoch
    int near_grid;          // launch size of the near part (an upper bound of the set's size)
    int* next_count;        // block 0 empties the next step's near list (it is filled by the particle phase)
    const uint32_t* step_in;  // device step counter of this buffer parity (dither of the half formats)
    uint32_t* step_out;       // the other parity's counter: set to step + 1 by block 0
    hipEvent_t ev_start;    // optional: events that receive the kernel's start and end timestamps
    hipEvent_t ev_stop;
};

// The near set: collide-stream blocks within a margin of some particle's
// window, updated by the particle stream while the far blocks run elsewhere.
struct NearSet {
    uint32_t* flags;        // one word per collide-stream block: epoch of the step it is near at
    int* list;              // block ids of the set
    int* count;
    uint32_t epoch;         // epoch this set is built for (step + 1)
    int rows_geom;          // 1: blocks are groups of 4 x-rows (row-wave kernel), 0: 256-site tiles
    int margin;             // nodes added on every side of the particle window
};

hipError_t launch_collide_stream(const LaunchCS& a, hipStream_t st);
hipError_t launch_init(const BoxDesc* boxes, const int* tile_box, int ntiles, void* f0, void* f1,
                       const int* box_init, const KParams& kp, hipStream_t st);
hipError_t launch_fields(const BoxDesc* boxes, int bi, const uint16_t* omap, const void* fin, int s0,
                         int count, double* out, const KParams& kp, hipStream_t st);
hipError_t launch_moments(const BoxDesc* boxes, int bi, int n, const uint16_t* omap, const void* fin,
                          double* partial, const KParams& kp, hipStream_t st);
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int blocks, hipStream_t st);
// Copies every population from its slot in convention cs (src) to its slot in
// convention cd (dst); src and dst are distinct buffers of the same layout.
hipError_t launch_relayout(const BoxDesc* boxes, const int* tile_box, int ntiles, const void* src, void* dst, int cs,
                           int cd, int storage, int q, hipStream_t st);
hipError_t launch_poke(const BoxDesc* boxes, int bi, void* f, int s, int dir, double val, const KParams& kp,
                       hipStream_t st);

struct LaunchPart {
    const BoxDesc* boxes;
    BoxRT* rt;
    PartDev* parts;
    uint32_t* links;
    uint16_t* omap;
    void* f;          // population buffer holding this step's post-collision values
    int* flags;
    int first, count; // particle range
    KParams kp;
    int lds_words;    // 32-bit words of the remap window bitmask
    int mode;         // remap: 0 step, 1 add (no transitions), 2 remove
    NearSet near;     // set of the next step: the preceding collide launch empties it, remap (mode 0) fills it
    // boxes with several particles (solve_map, claim, links):
    uint32_t* stamps;        // per cell of 8^3 nodes: the epoch of the last step an owner changed there
    const uint32_t* epoch;   // this step's epoch (the device step counter after the collide launch)
    uint32_t* cand;          // claim candidates, lds_words bit words per particle
    int force_box;           // links: >= 0 rebuild every particle of this box (set-up), else -1
    uint32_t* band;          // narrow band of each particle's last full scan, lds_words bit words per particle
    int use_band;            // rescans within the band test only its nodes (0: every scan is full)
};

hipError_t launch_particle_remap(const LaunchPart& a, hipStream_t st);
hipError_t launch_particle_step(const LaunchPart& a, hipStream_t st);  // solve + remap, one particle per box
// boxes with several particles: the three kernels of a step, in this order
hipError_t launch_particle_solve_map(const LaunchPart& a, hipStream_t st);
hipError_t launch_particle_claim(const LaunchPart& a, hipStream_t st);
hipError_t launch_particle_links(const LaunchPart& a, hipStream_t st);
size_t particle_remap_lds_bytes(int lds_words);
hipError_t launch_near_mark(const LaunchPart& a, hipStream_t st);

// ---- warm-start surrogate: 8 -> 64 -> 64 -> 6 tanh MLP (k_mlp.hip) ----
constexpr int MLP_IN = 8, MLP_H = 64, MLP_OUT = 6;
// flat parameters: W1[64][8], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]
constexpr int MLP_OW1 = 0, MLP_OB1 = MLP_OW1 + MLP_H * MLP_IN, MLP_OW2 = MLP_OB1 + MLP_H,
              MLP_OB2 = MLP_OW2 + MLP_H * MLP_H, MLP_OW3 = MLP_OB2 + MLP_H, MLP_OB3 = MLP_OW3 + MLP_OUT * MLP_H,
              MLP_NP = MLP_OB3 + MLP_OUT;

struct MlpArgs {
    const float* P;   // FP32 parameters
    const float* X;   // n x 8 inputs
    const float* Y;   // n x 6 targets (mode 1)
    float* out;       // n x 6 outputs (mode 0)
    float* G;         // per-tile partial gradients, ceil(n / 16) x MLP_NP (mode 1)
    float* Lpart;     // per-tile sums of squared errors (mode 1)
    int n;
    float scale;      // dL/dy = scale * (y - Y)
    int mode;         // 0 forward, 1 forward + backward
};
struct MlpReduceArgs {
    const float* G;
    const float* Lpart;
    int ntiles;
    float* P;
    float* M;
    float* V;
    float lr, c1, c2;  // Adam: step size, 1 / (1 - beta1^t), 1 / (1 - beta2^t)
    float* gsum;       // mode 1: summed gradient
    double* loss_acc;  // += sum of the tiles' squared errors (may be null)
    float* loss_out;   // or: = that sum / loss_div (may be null)
    double loss_div;
    int mode;          // 0 Adam update, 1 write the summed gradient
};
hipError_t launch_mlp(const MlpArgs& a, hipStream_t st);
hipError_t launch_mlp_reduce(const MlpReduceArgs& a, hipStream_t st);

// ---- warm start (k_warm.hip) ----
hipError_t launch_warm_features(const BoxDesc* boxes, const PartDev* parts, int np, double mu, float* X, double* s,
                                hipStream_t st);
hipError_t launch_warm_apply(PartDev* parts, int np, const float* Y, const double* s, double mu, double* pred,
                             int only_box, hipStream_t st);
hipError_t launch_warm_targets(const PartDev* parts, int np, const double* s, double mu, float* Y, hipStream_t st);
size_t stokes_scratch_doubles(int nboxes, int ntiles);  // scratch of launch_stokes_start
int stokes_free_doubles();  // doubles per node of its staged free field (uf)
// only_box >= 0: that box only (every box otherwise).  uf: stokes_free_doubles()
// doubles per node of the started boxes, node (box B, site s) at that many
// times (B.ooff + s - base).
hipError_t launch_stokes_start(const BoxDesc* boxes, int nboxes, const int* tile_box, int ntiles,
                               const uint16_t* omap, const PartDev* parts, int np, double mu, double* scratch,
                               double* uf, long long base, void* f, const KParams& kp, int only_box, hipStream_t st);
// ---- fallback monitor of warm-started boxes ----
// per tile: sum over fluid sites of |j|^2 for boxes whose monitor is pending (k_stream.hip)
hipError_t launch_box_energy(const BoxDesc* boxes, const int* tile_box, int ntiles, const uint16_t* omap,
                             const void* fin, const BoxMon* mon, double* partial, const KParams& kp, hipStream_t st);
// one work-group per box: residuals, decision, particle reset; then the populations of boxes that fell back
hipError_t launch_warm_monitor(const BoxDesc* boxes, int nboxes, const int* tile_box, int ntiles, BoxMon* mon,
                               const double* partial, PartDev* parts, int np, const double* pred, double* vref,
                               long long step, void* f, int storage, int q, hipStream_t st);

}  // namespace lbd
