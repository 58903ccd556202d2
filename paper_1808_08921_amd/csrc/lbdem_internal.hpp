// lbdem_internal.hpp -- device-side data layout shared by the kernels and the host API.
//
// All device buffers of a set are carved out of one workspace.  Fields are SoA with x
// fastest.  Populations are double-buffered (A/B) and the node map, the particle state
// and the node-change list are double-buffered by the parity of the step counter that
// lives in device memory, so that a fixed sequence of kernel launches (a HIP graph)
// advances the set without host involvement.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbdem {

constexpr int kQ = 19;
constexpr int kWaveSlots = 12;     // link-force partial slots per wavefront tile
constexpr int kNearCap = 32;       // near-neighbour table per particle
constexpr int kHistCap = 16;       // tangential contact history per particle
constexpr double kNearMargin = 3.0; // near list: |X_p - X_q| <= R_p + R_q + margin
constexpr double kShell = 0.5;      // skin of the per-particle shell lists (lattice units)
constexpr int kChunks = 8;          // workgroups per particle in the particle kernel
constexpr int kEmpty = 0x7fffffff;

// Per-lattice constants (one entry per lattice of the set).
struct MemberDev {
    int nx, ny, nz;
    int bx_log2, bx, by;      // tile extent in x (power of two) and y; bx*by = 256
    int ntx, nty, ntz;        // tiles per axis
    int tile_off;             // first global tile index of this lattice
    int bc[6];                // face kinds
    int per[3];               // periodic axes
    double box[3];            // axis lengths as doubles
    long long ncell;          // nx*ny*nz
    long long cell_off;       // offset of this lattice in node-map arrays
    long long pop_off;        // offset of this lattice in population arrays (19*cell_off)
    double omega;             // 1/tau
    double rho_f;
    long long wave_off;       // offset in the waveform table (t_n + 2 entries)
    long long t_n;
    int pz_off;               // offset in the z -> probe-index map (nz entries)
    int plist_off;            // offset in the probe-plane list (n_probe entries)
    int n_probe;
    long long ring_off;       // offset (doubles) of this lattice's probe ring
    int p_off, p_cap, np;     // particles: global offset, capacity, current count
    double E, nu, mu, rho_p;
};

// Everything a kernel needs, passed by value.
struct DevSet {
    int nmem;
    const MemberDev *mem;
    int tiles_total;
    int nzt;                  // z planes per fluid-kernel thread
    // populations
    void *popA, *popB;
    // node maps (index = parity), change lists (pairs cell, owner) and counts
    int *own[2];
    int *chg[2];
    int chg_cap;
    int *chgcnt;              // [2]
    // probes
    double *pprt;             // [tiles_total*nzt*4]
    double *ring;
    int ring_len;
    const short *pzmap;
    const int *plist;
    int nprobe_total;
    const double *wave;
    // particles
    int ptot;
    double *X[2], *V[2], *W[2];
    double *R, *m, *I, *Fg, *Fh, *Th, *Ph, *Lh, *Xref, *margin;
    int *fixed, *pmem;
    double *ppart;            // link-force partials per (particle, chunk) [ptot*kChunks*6]
    int *nearl, *nnear;       // [ptot*kNearCap], [ptot]
    // shell list per particle around X_ref: node, d_ref - R, link-candidate directions
    int lcap;
    int *lcell, *lcnt;
    float *ldr;
    unsigned *lmask;
    int *hj[2];               // tangential history partner ids [ptot*kHistCap]
    double *hf[2];            // tangential history forces [ptot*kHistCap*3]
    int *hn[2];               // history counts [ptot]
    // counters
    long long *tstep;         // steps completed
    long long *tcopy;         // step in progress, for the re-projection kernel
    unsigned int *flags;
};

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_PRESSURE = 2 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16DEV = 2, PREC_BF16DEV = 3 };

// kernel launchers (lbdem_kernels.hip)
hipError_t launch_links(int prec, const DevSet &s, hipStream_t st);
hipError_t launch_motion(const DevSet &s, int mode, int only_member, hipStream_t st);
hipError_t launch_fluid(int prec, const DevSet &s, hipStream_t st);
hipError_t launch_remap_prec(int prec, const DevSet &s, int mode, int only_member, hipStream_t st);
hipError_t launch_init_pops(int prec, const DevSet &s, long long total_cells, hipStream_t st);
// kernel entry points and grid sizes, for building HIP graphs
void *links_kernel_ptr(int prec);
void *motion_kernel_ptr();
void *fluid_kernel_ptr(int prec);
void *remap_kernel_ptr_prec(int prec);
int links_grid(const DevSet &s);
int motion_grid(const DevSet &s);
int remap_grid(const DevSet &s);

} // namespace lbdem
