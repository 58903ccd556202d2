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
constexpr int kNearCap = 32;       // near-neighbour table per particle
constexpr int kHistCap = 16;       // tangential contact history per particle
constexpr double kNearMargin = 3.0; // near list: |X_p - X_q| <= R_p + R_q + margin
constexpr int kNearEvery = 5;       // steps between near-list builds (approach < 0.5 lu per step)
constexpr double kShell = 0.5;      // skin of the per-particle shell lists (lattice units)
constexpr double kBandIn = 0.15;    // surface band list: nodes with -kBandIn <= d - R <= kBandOut
constexpr double kBandOut = 0.1;    // (lattice units)
// node lists keep the solid nodes within a skin of a surface; the skin of a rebuild is
// kSkinSteps times the largest particle step of the lattice, within [kSkinMin, kListSkin]
constexpr double kListSkin = 0.25;
constexpr double kSkinMin = 0.05;
constexpr double kSkinSteps = 12.0;
constexpr int kPendCap = 16384;     // refills of unlisted nodes awaiting the next list rebuild
constexpr int kChunks = 8;          // chunks of a shell list: waves per particle in the link pass
// components of a link-pass partial per (particle, chunk): F0 (3) and sum xr x G (3), xr the
// node position relative to the shell list's reference point
constexpr int kLinkComp = 6;
// cached link-set sums per (particle, chunk): S (6, upper triangle), Qx (9, row-major), Wx (6)
constexpr int kZComp = 21;
constexpr int kEmpty = 0x7fffffff;
// Link words of a fluid node x (two 64-bit words per node: lw[c] and lw[ncell_total + c]).
// Word 0: bits 0-17 the directions e whose source x - c_e is inside a particle, bits 18-35
// the low bit of the slot (0..3) of the particle owning that source, bits 36-48 and 49-61
// the local indices of the particles in slots 0 and 1, bit 62 set when slots 2 or 3 are
// used, bit 63 when more than four particles border x.  Word 1: bits 0-17 the high slot
// bit per direction, bits 18-30 and 31-43 the local indices in slots 2 and 3.
constexpr int kMaxLocal = 8191;     // particles per lattice (13-bit local indices)
constexpr int kRefreshBlocks = 512; // workgroups of the start-of-step refresh kernel
constexpr int kMaxPlaneWords = 8192; // row-table words of one x-y plane held in LDS (compact storage)
constexpr int kRtLds = 1536;        // row-table words a fluid-kernel workgroup stages in LDS (compact storage)

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
    int nw;                   // 32-node words per x row (compact storage)
    long long rt_off;         // offset of this lattice's row tables (compact storage)
    long long pv_from;        // first step whose particle velocities the ring holds for this lattice
    // 1: a periodic axis shorter than 2 max_radius + 4, where a fluid node can have links
    // into two images of one particle; its links are then grouped per (particle, image)
    // and the arm of a group is taken from the midpoint of one of its links
    int narrow;
    int rest_free;            // 1: link forces without the rest state's part (lbdem_params.rest_free)
};

// Everything a kernel needs, passed by value.
struct DevSet {
    int nmem;
    int fluid_off;            // 1: hydrodynamics switched off (particles feel contacts and F_g only)
    int narrow;               // 1: some lattice of the set is narrow (MemberDev::narrow)
    const MemberDev *mem;
    int tiles_total;
    int nzt;                  // z planes per fluid-kernel thread
    // node lists: per lattice and z plane, the listed nodes in x-fastest order at
    // [cell_off + z*nx*ny, +count); the fluid kernel then runs one thread per listed node
    int listmode;
    // compact storage (with node lists): populations of the listed nodes of plane z at
    // slots z*nx*ny + rank (rank in list order); row tables give, per x row and 32-node
    // word, the listed-node bits and the rank of the word's first listed node
    int compact;
    int es;                   // bytes per stored population value
    uint2 *rt;                // [sum over lattices of nz*ny*nw]
    void *popC;               // scratch population buffer for re-layouts
    int nplanes;              // sum of nz over the lattices
    int *clist;               // [ncell_total]
    int *ccnt;                // [sum of nz], indexed like the z -> probe map
    double *Xl;               // particle positions when the lists were built [ptot*3]
    long long *relist_at;     // step whose refresh rebuilds the lists
    double *skin;             // skin of each lattice's current lists [nmem]
    double list_margin;       // look-ahead of the rebuild trigger, in particle steps
    double *pspd;             // each particle's displacement in its last step [ptot]
    // compact storage: a node uncovered outside the lists has its refill (rho_bar, V_b)
    // parked until the next step's list rebuild: record index per node (-1 none)
    // [ncell_total], records [2][kPendCap*4] and counts [2] by the parity of the step
    int *pend;
    double *pbuf[2];
    int *pcnt;
    // populations
    void *popA, *popB;
    // node maps (index = parity), change lists (pairs cell, owner) and counts
    int *own[2];
    unsigned long long *lw;   // link words, two per node (all lattices) [2*ncell_total]
    // compact storage: the first link word of each listed node at its storage slot, or
    // kSolidWord for a listed solid node (the fluid and record kernels read these in slot
    // order), and the step at which a full copy of the node map made them all stale
    unsigned long long *lwc;  // [ncell_total]
    long long *lwc_bad;
    long long ncell_total;
    // per slot of a fluid node's link words, written by k_records of step t for the link
    // pass of step t: G = sum c_d (f~_d(x,t) - w_d rho_f) over the slot's links and the link
    // directions (FP32 float4, FP64 two double2), [4][ncell_total] at the node's storage
    // slot; rec_step: the step whose k_records wrote them
    void *frec;
    long long *rec_step;
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
    float *pf[2];             // FP32 wall state of the fluid kernel per particle (12 floats): X(t) and the
                              // velocities V, Omega of step t, at the parity of t
    int *fixed, *pmem;
    double *pvring;           // particle velocities after each step [pv_ring][ptot][3] (0 steps: none)
    int pv_ring;
    double *ppart;            // link-pass partials per (particle, chunk) [ptot*kChunks*kLinkComp]
    double *zcache;           // link-set sums per (particle, chunk), rebuilt with its entries [ptot*kChunks*kZComp]
    int *nearl, *nnear;       // [ptot*kNearCap], [ptot]
    long long *near_at;       // step at which each near list was built [ptot]
    // shell list per particle around X_ref: node, d_ref - R, link-candidate directions
    int lcap;
    int *lcell, *lcnt;
    float *ldr;
    unsigned *lmask;
    // the shell-list entries that hold links of the particle: each chunk of a list keeps
    // its own compacted run [ptot*lcap], counts [ptot*kChunks]
    int *xcell, *xcnt;
    int *xslot;               // storage slot of each cached entry's node [ptot*lcap]
    unsigned *xgrp;           // the particle's link directions at each cached entry's node [ptot*lcap]
    long long *lreb;          // step after which the shell list was last rebuilt [ptot]
    long long *ldirty;        // last step in which a node of a chunk's z-slab, or next to
                              // it, changed owner [ptot*kChunks]
    // chunks are z-slabs of the list's scan box: first z (unwrapped), slab height, and
    // the list offset where each chunk starts [ptot*2], [ptot*(kChunks+1)]
    int *lzr, *lchunk;
    // running maxima since the last shell-list rebuild of |X - X_ref| and of |X - X_ref|
    // plus the overlap depth with the near neighbours [ptot] each
    double *rdisp, *rlens;
    // surface band: shell-list entries with -kBandIn <= d_ref - R <= kBandOut [ptot*bcap], [ptot]
    int bcap;
    int *bcell, *bcnt;
    float *bdr;
    int *hj[2];               // tangential history partner ids [ptot*kHistCap]
    double *hf[2];            // tangential history forces [ptot*kHistCap*3]
    int *hn[2];               // history counts [ptot]
    // counters
    long long *tstep;         // steps completed
    long long *tcopy;         // step in progress, for the re-projection kernel
    unsigned int *flags;
};

// Adjoint window over frozen geometry (one lattice): device view.
struct AdjDev {
    MemberDev M;              // the lattice's constants (offsets relative to this lattice)
    int ncell;
    const int *own;           // frozen node map, local particle indices [ncell]
    const double *X, *W, *R;  // particle positions, angular velocities [np*3], radii [np]
    const double *V;          // particle velocities of the window [np*3]
    int np;
    double rho_f, omega, amp; // omega = 1/tau and the waveform amplitude of the window
    const double *shape;      // unit-amplitude waveform at time level t0+n+1 [nsteps]
    int n_probe;
    const int *probe_z;       // [n_probe]
    const double *probe_nfl;  // fluid nodes per probe plane [n_probe]
    double *P;                // probe signals [nsteps][n_probe]
    const double *dLdP;       // loss gradient [nsteps][n_probe]
    double *acc_w, *acc_a;    // per-workgroup sums of dL/domega and dL/dA [nblk]
    double *macc;             // summed dL/dg of every direction whose source is a particle [18][ncell]
    double *gv;               // dL/dV [np*3]
};

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_PRESSURE = 2 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16DEV = 2, PREC_BF16DEV = 3 };

// kernel launchers (lbdem_kernels.hip)
hipError_t launch_refresh(int prec, const DevSet &s, hipStream_t st);
hipError_t launch_records(int prec, const DevSet &s, hipStream_t st);
hipError_t launch_links(int prec, const DevSet &s, hipStream_t st);
hipError_t launch_motion(const DevSet &s, int mode, int only_member, hipStream_t st);
hipError_t launch_fluid(int prec, const DevSet &s, hipStream_t st);
hipError_t launch_remap_prec(int prec, const DevSet &s, int mode, int only_member, hipStream_t st);
hipError_t launch_init_pops(int prec, const DevSet &s, long long total_cells, hipStream_t st);
hipError_t launch_expand(int prec, const DevSet &s, hipStream_t st);
hipError_t launch_fields(int prec, const DevSet &s, int m, long long ncell, double *out, hipStream_t st);
// kernel entry points and grid sizes, for building HIP graphs
void *refresh_kernel_ptr(int prec);
void *records_kernel_ptr(int prec, int compact, int narrow);
int records_grid(const DevSet &s);
void *links_kernel_ptr(int prec, int narrow);
void *motion_kernel_ptr();
void *fluid_kernel_ptr(int prec, int compact, int narrow);
void *remap_kernel_ptr_prec(int prec);
int refresh_grid(const DevSet &s);
int links_grid(const DevSet &s);
int links_block();
int motion_grid(const DevSet &s);
int remap_grid(const DevSet &s);
// adjoint window kernels (lbdem_kernels.hip)
hipError_t launch_adj_step(int prec, const AdjDev &a, const void *fin, void *fout, int n, hipStream_t st);
hipError_t launch_adj_probe(int prec, const AdjDev &a, const void *fin, int n, hipStream_t st);
hipError_t launch_adj_mu(int prec, const AdjDev &a, const void *fin, const void *lam, void *mu, int n, hipStream_t st);
hipError_t launch_adj_pull(int prec, const AdjDev &a, const void *mu, void *lam, hipStream_t st);
hipError_t launch_adj_vgrad(const AdjDev &a, hipStream_t st);
hipError_t launch_adj_nfl(const AdjDev &a, double *nfl, hipStream_t st);
int adj_blocks(const AdjDev &a);


// dispersion analysis (lbdem_analysis.hip)
struct DftPlan {
    int nwb, nzb, threads, nchunk;   // frequency blocks of 64, column blocks, threads per block, time chunks
    long long chunk;                  // steps per time chunk
    size_t part_bytes, g_bytes, e_bytes;  // workspace: chunk partials, time-stage sums, phase table
};
DftPlan dft_plan(long long nt, int nz, int nw, int nk);
hipError_t launch_st_dft(const DftPlan &p, const double *x, long long nt, int nz, const double *zpos, double t0,
                         double w0, double dw, int nw, double k0, double dk, int nk, double *F, int *ridge,
                         void *work, hipStream_t st);
hipError_t launch_wave_fit(const double *x, long long nt, int nz, const double *zpos, double t0, double omega,
                           double *out, void *work, hipStream_t st);
// the allocation-free fit's static device scratch: its size, and its address on the
// current device (looked up once per device)
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
hipError_t noalloc_scratch(void **ptr);
hipError_t launch_particle_signal(const double *ring, int ring_len, int ptot, int p_off, long long first,
                                  long long n, const int *start, const int *members, int n_layers, int component,
                                  double *x, hipStream_t st);
hipError_t launch_probe_signal(const double *ring, int ring_len, int nprobe, long long first, long long n,
                               int quantity, double *x, hipStream_t st);

} // namespace lbdem
