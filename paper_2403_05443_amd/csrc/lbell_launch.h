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
};

hipError_t launch_collide_stream(const LaunchCS& a, hipStream_t st);
hipError_t launch_init(const BoxDesc* boxes, const int* tile_box, int ntiles, void* f0, void* f1,
                       const int* box_init, const KParams& kp, hipStream_t st);
hipError_t launch_fields(const BoxDesc* boxes, int bi, const uint16_t* omap, const void* fin, int s0,
                         int count, double* out, const KParams& kp, hipStream_t st);
hipError_t launch_moments(const BoxDesc* boxes, int bi, int n, const uint16_t* omap, const void* fin,
                          double* partial, const KParams& kp, hipStream_t st);
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
};

hipError_t launch_particle_solve(const LaunchPart& a, hipStream_t st);
hipError_t launch_particle_remap(const LaunchPart& a, hipStream_t st);
size_t particle_remap_lds_bytes(int lds_words);

}  // namespace lbd
