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
    int spt;                // generic tiles: 256-site tiles per block (1 or 2)
    bool xcd;               // generic tiles: XCD-chunked block order
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
};

hipError_t launch_particle_solve(const LaunchPart& a, hipStream_t st);
hipError_t launch_particle_remap(const LaunchPart& a, hipStream_t st);
hipError_t launch_particle_step(const LaunchPart& a, hipStream_t st);  // solve + remap, one particle per box
size_t particle_remap_lds_bytes(int lds_words);
hipError_t launch_near_mark(const LaunchPart& a, hipStream_t st);

}  // namespace lbd
