// lbdem_kernels.hip -- gfx950 kernels of the coupled lattice-Boltzmann / DEM step.
//
// Method: Cheng, Luding, Rivas, Harting, Magnanimo, "Hydro-micromechanical modeling of
// wave propagation in saturated granular media", arXiv 1808.08921, Sec. 2.
//
// Six kernels make one time step t -> t+1 of every lattice of a set, in this order
// (Secs. 2.1-2.4; the paper gives no order: this one lets the particle velocities of the
// step be solved together with the momentum their links exchange in it):
//   k_refresh    brings the node map of step t up to date with the previous re-projection's
//                changes, refreshes the link words of the changed nodes and their
//                neighbours, and rebuilds the node lists (moving the populations of changed
//                planes under compact storage) once a particle may have crossed their skin.
//   k_records    first kChunks waves per particle, rebuilding the link entries of the
//                chunks of its shell list whose link words changed, with their link-set
//                sums (the 6 x 6 matrix Z of the motion kernel comes from them); then one
//                thread per listed node (or node of a dense tile): per link slot of a fluid
//                node, the sum of c_d (f~_d(x,t) - w_d rho_f) over the slot's links.
//   k_links      kChunks waves per particle: the link pass.  With Eq. (mem) substituted, the
//                link force of Eq. (fFS) is 2 c_d f~_d(x,t) minus a term linear in the
//                particle's velocities; per (particle, chunk) the first part and its torque
//                (F0, T0) are summed in FP64 from the records of f~(t).
//   k_motion     one wave per particle: contacts (Eqs. fdLawn, fdLaws) at X(t), then the
//                velocities of the step from (M + Z)(V', Omega') = M (V, Omega) + F0 + contacts
//                + F_g + the conversion impulses of the previous re-projection (Eqs. translate,
//                rotate, coupleF, coupleT; implicit in the exchanged momentum), X(t+1).
//   k_fluid      one thread per listed node of a z plane (compact storage, the default), or
//                per node of a dense tile: pull streaming (Eq. stream) with stationary walls,
//                moving half-way bounce-back at the particles' new velocities (Eq. mem), the
//                density faces (Sec. 2.4), BGK collision (Eqs. bgk, BGKequili, rhoAndU) and
//                probe partial sums.
//   k_remap      one wave per particle: re-projects the particle on the lattice (Sec. 2.3)
//                where its motion can have changed a node, converts covered and uncovered
//                nodes (Eqs. convertFS, convertSF) and records the impulses that act in the
//                next step; extra workgroups reduce the probe planes; the step counter
//                advances.
// Populations are SoA, [19][nz][ny][nx] per lattice in the node layout, or per z plane at
// the ranks of the plane's listed nodes under compact storage.  The fluid kernel is bound
// by HBM bandwidth (about 1.5 flop per byte at FP32) and uses no MFMA.
#include "lbdem_internal.hpp"

namespace lbdem {

// D3Q19 velocity set in the paper's order (Eq. 3d19q); index = paper index - 1.
constexpr int kCX[kQ] = {1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
constexpr int kCY[kQ] = {0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
constexpr int kCZ[kQ] = {0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};
constexpr int kOPP[kQ] = {1, 0, 3, 2, 5, 4, 11, 10, 13, 12, 7, 6, 9, 8, 17, 16, 15, 14, 18};
// the same components in device memory, for a direction known only at run time
__constant__ int kCXd[kQ] = {1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
__constant__ int kCYd[kQ] = {0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
__constant__ int kCZd[kQ] = {0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};
// lattice weights (Sec. 2.1): 1/18 along the axes, 1/36 on the diagonals, 1/3 at rest
constexpr double kWd[kQ] = {1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 3};
constexpr double kCS2 = 1.0 / 3.0;
// 2 w_d / c_s^2 of the moving-wall term of Eq. (mem)
constexpr double kMW[kQ] = {2.0 * kWd[0] / kCS2, 2.0 * kWd[1] / kCS2, 2.0 * kWd[2] / kCS2, 2.0 * kWd[3] / kCS2,
                            2.0 * kWd[4] / kCS2, 2.0 * kWd[5] / kCS2, 2.0 * kWd[6] / kCS2, 2.0 * kWd[7] / kCS2,
                            2.0 * kWd[8] / kCS2, 2.0 * kWd[9] / kCS2, 2.0 * kWd[10] / kCS2, 2.0 * kWd[11] / kCS2,
                            2.0 * kWd[12] / kCS2, 2.0 * kWd[13] / kCS2, 2.0 * kWd[14] / kCS2, 2.0 * kWd[15] / kCS2,
                            2.0 * kWd[16] / kCS2, 2.0 * kWd[17] / kCS2, 2.0 * kWd[18] / kCS2};
// 1 / w_d (exact) for the 16-bit deviation codec
constexpr float kInvW[kQ] = {18, 18, 18, 18, 18, 18, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 3};

// ---------------------------------------------------------------------------
// storage precisions
// ---------------------------------------------------------------------------
template <int P> struct Prec;
template <> struct Prec<PREC_FP64> { using S = double; using C = double; };
template <> struct Prec<PREC_FP32> { using S = float; using C = float; };
template <> struct Prec<PREC_FP16DEV> { using S = _Float16; using C = float; };
template <> struct Prec<PREC_BF16DEV> { using S = uint16_t; using C = float; };

__device__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u); // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// element idx of an array whose byte size stays below 4 GiB: a 32-bit byte offset from a
// base that is the same in every lane (scalar base + vector offset addressing)
template <typename T>
__device__ __forceinline__ T ldo(const T *base, unsigned idx)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void sto(T *base, unsigned idx, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (unsigned)sizeof(T)) = v;
}

// decode population d from storage: FP64 holds f, FP32 the deviation f - w_d rho_f (the
// rest value rounded once to FP32), the 16-bit forms q = f / w_d - rho_f
template <int P>
__device__ __forceinline__ typename Prec<P>::C ld(const typename Prec<P>::S *a, unsigned idx, int d, double rho_f)
{
    if constexpr (P == PREC_FP64) {
        return ldo(a, idx);
    } else if constexpr (P == PREC_FP32) {
        return ldo(a, idx) + (float)(kWd[d] * rho_f);
    } else if constexpr (P == PREC_FP16DEV) {
        return (float)kWd[d] * ((float)rho_f + (float)ldo(a, idx));
    } else {
        return (float)kWd[d] * ((float)rho_f + bf16_to_f32(ldo(a, idx)));
    }
}
// encode population d to storage
template <int P>
__device__ __forceinline__ void st(typename Prec<P>::S *a, unsigned idx, int d, typename Prec<P>::C f, double rho_f)
{
    using S = typename Prec<P>::S;
    if constexpr (P == PREC_FP64) {
        sto(a, idx, (S)f);
    } else if constexpr (P == PREC_FP32) {
        sto(a, idx, f - (float)(kWd[d] * rho_f));
    } else if constexpr (P == PREC_FP16DEV) {
        sto(a, idx, (S)(f * kInvW[d] - (float)rho_f));
    } else {
        sto(a, idx, f32_to_bf16(f * kInvW[d] - (float)rho_f));
    }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_swizzle(int b, int G)
{
    // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous tile range
    const int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

__device__ __forceinline__ double mimg(double dx, int per, double n)
{
    if (per) {
        if (dx > 0.5 * n) dx -= n;
        else if (dx < -0.5 * n) dx += n;
    }
    return dx;
}

// Position of fluid node (i, j, k) relative to the image of a particle centre X that holds
// the node's link group grp (directions e whose source x - c_e lies in that image): the
// minimum image of x - X, or, in a set with a narrow periodic lattice (NR), where two
// images can border one node, the minimum image of the first link's midpoint x - c_e / 2
// (always less than half a period from its own image's centre) plus c_e / 2.
template <bool NR>
__device__ __forceinline__ void group_arm(const MemberDev *M, unsigned grp, int i, int j, int k, double X0, double X1,
                                          double X2, double &r0, double &r1, double &r2)
{
    if constexpr (NR) {
        const int e = __ffs(grp) - 1;
        const double h0 = 0.5 * (double)kCXd[e], h1 = 0.5 * (double)kCYd[e], h2 = 0.5 * (double)kCZd[e];
        r0 = mimg(((double)i - h0) - X0, M->per[0], M->box[0]) + h0;
        r1 = mimg(((double)j - h1) - X1, M->per[1], M->box[1]) + h1;
        r2 = mimg(((double)k - h2) - X2, M->per[2], M->box[2]) + h2;
    } else {
        r0 = mimg((double)i - X0, M->per[0], M->box[0]);
        r1 = mimg((double)j - X1, M->per[1], M->box[1]);
        r2 = mimg((double)k - X2, M->per[2], M->box[2]);
    }
}

// Image of particle centre X (per axis -1, 0 or +1 periods, packed 2 bits an axis) that
// holds the source (si, sj, sk) of a link, given unwrapped (it may lie one node outside
// the lattice); 0 on a lattice that is not narrow.
__device__ __forceinline__ int source_image(const MemberDev *M, int si, int sj, int sk, const double *X)
{
    if (!M->narrow) return 0;
    const int s3[3] = {si, sj, sk};
    int code = 0;
    for (int a = 0; a < 3; ++a) {
        int n = 0;
        if (M->per[a]) {
            const double d = (double)s3[a] - X[a];
            n = (d > 0.5 * M->box[a]) ? 1 : (d < -0.5 * M->box[a]) ? -1 : 0;
        }
        code |= (n + 1) << (2 * a);
    }
    return code;
}

__device__ __forceinline__ double dist2(const MemberDev *M, int i, int j, int k, double X0, double X1, double X2)
{
    const double dx = mimg((double)i - X0, M->per[0], M->box[0]);
    const double dy = mimg((double)j - X1, M->per[1], M->box[1]);
    const double dz = mimg((double)k - X2, M->per[2], M->box[2]);
    return (dx * dx + dy * dy) + dz * dz;
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i(int v, int old)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xf, false);
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes in a fixed order, returned to every lane: DPP sums within each
// row of 16 lanes, then the four row sums are added in row order.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_d<0xB1, 0xF>(v);  // quad_perm [1,0,3,2]
    v += dpp_d<0x4E, 0xF>(v);  // quad_perm [2,3,0,1]
    v += dpp_d<0x141, 0xF>(v); // row_half_mirror
    v += dpp_d<0x140, 0xF>(v); // row_mirror
    return ((readlane_d(v, 0) + readlane_d(v, 16)) + readlane_d(v, 32)) + readlane_d(v, 48);
}
__device__ __forceinline__ int wave_sum_i(int v)
{
    v += dpp_i<0xB1, 0xF>(v, 0);
    v += dpp_i<0x4E, 0xF>(v, 0);
    v += dpp_i<0x141, 0xF>(v, 0);
    v += dpp_i<0x140, 0xF>(v, 0);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}
// Minimum over the 64 lanes, returned to every lane.
__device__ __forceinline__ int wave_min(int v)
{
    v = min(v, dpp_i<0xB1, 0xF>(v, v));
    v = min(v, dpp_i<0x4E, 0xF>(v, v));
    v = min(v, dpp_i<0x141, 0xF>(v, v));
    v = min(v, dpp_i<0x140, 0xF>(v, v));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ double wave_min_d(double v)
{
    // values are non-negative here: the bit patterns order like the values
    long long b = __double_as_longlong(v);
    int hi = (int)(b >> 32);
    unsigned lo = (unsigned)b;
    for (int off = 32; off >= 1; off >>= 1) {
        const int ohi = __shfl_xor(hi, off, 64);
        const unsigned olo = (unsigned)__shfl_xor((int)lo, off, 64);
        if (ohi < hi || (ohi == hi && olo < lo)) { hi = ohi; lo = olo; }
    }
    return __longlong_as_double(((long long)hi << 32) | lo);
}

// Block-wide (256 threads) sums of N doubles in a fixed order; result valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*red)[8])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < N; ++c) red[wv][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < N; ++c) v[c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    __syncthreads();
}

// values that are the same in every lane, moved to scalar registers
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni(long long v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double uni(double v) { return __longlong_as_double(uni((long long)__double_as_longlong(v))); }

__device__ __forceinline__ const MemberDev *member_of_tile(const DevSet &s, int g)
{
    int lo = 0, hi = s.nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.mem[mid].tile_off <= g) lo = mid;
        else hi = mid - 1;
    }
    return s.mem + uni(lo);
}

__device__ __forceinline__ int wrap_axis(int c, int n, int bclo, int bchi, int &kind)
{
    if (c < 0) { kind = max(kind, bclo); return c + n; }
    if (c >= n) { kind = max(kind, bchi); return c - n; }
    return c;
}

// Density boundary on a z face: non-equilibrium bounce-back (Sec. 2.4) with zero
// tangential velocity; the velocity normal to the face follows from the density.
template <typename C>
__device__ __forceinline__ void zou_he(C (&f)[kQ], C rho, bool top)
{
    // paper indices k -> f[k-1]
    const C s0 = f[0] + f[1] + f[2] + f[3] + f[6] + f[7] + f[10] + f[11] + f[18];
    const C nxc = C(0.5) * (f[0] + f[6] + f[7] - f[1] - f[10] - f[11]);
    const C nyc = C(0.5) * (f[2] + f[6] + f[10] - f[3] - f[7] - f[11]);
    if (!top) {
        const C sm = f[5] + f[9] + f[13] + f[15] + f[17];
        const C ruz = rho - (s0 + C(2) * sm);
        f[4] = f[5] + ruz / C(3);
        f[8] = f[13] + ruz / C(6) - nxc;
        f[12] = f[9] + ruz / C(6) + nxc;
        f[14] = f[17] + ruz / C(6) - nyc;
        f[16] = f[15] + ruz / C(6) + nyc;
    } else {
        const C sp = f[4] + f[8] + f[12] + f[14] + f[16];
        const C ruz = (s0 + C(2) * sp) - rho;
        f[5] = f[4] - ruz / C(3);
        f[13] = f[8] - ruz / C(6) + nxc;
        f[9] = f[12] - ruz / C(6) - nxc;
        f[17] = f[14] - ruz / C(6) + nyc;
        f[15] = f[16] - ruz / C(6) - nyc;
    }
}

// acc + sign * v, or sign * v when acc holds no term yet (a sum started from 0 would keep
// an addition of 0 that IEEE signed zeros do not let the compiler drop)
template <typename C>
__device__ __forceinline__ void acc_term(C &acc, bool &any, int sign, C v)
{
    if (sign == 0) return;
    if (any) acc = (sign > 0) ? acc + v : acc - v;
    else acc = (sign > 0) ? v : -v;
    any = true;
}

// c_d . u
template <typename C>
__device__ __forceinline__ C cdot(int d, C ux, C uy, C uz)
{
    C cu = C(0);
    bool any = false;
    acc_term(cu, any, kCX[d], ux);
    acc_term(cu, any, kCY[d], uy);
    acc_term(cu, any, kCZ[d], uz);
    return cu;
}

// rho = sum f, j = sum f c (Eq. rhoAndU), summed in direction order
template <typename C>
__device__ __forceinline__ void moments(const C (&f)[kQ], C &rho, C &jx, C &jy, C &jz)
{
    C r = C(0), x = C(0), y = C(0), z = C(0);
    bool ar = false, ax = false, ay = false, az = false;
#pragma unroll
    for (int d = 0; d < kQ; ++d) {
        acc_term(r, ar, 1, f[d]);
        acc_term(x, ax, kCX[d], f[d]);
        acc_term(y, ay, kCY[d], f[d]);
        acc_term(z, az, kCZ[d], f[d]);
    }
    rho = r; jx = x; jy = y; jz = z;
}

// f^eq_d(rho, u), Eq. (BGKequili)
template <typename C>
__device__ __forceinline__ C feq(int d, C rho, C ux, C uy, C uz, C uu)
{
    const C cu = cdot(d, ux, uy, uz);
    if constexpr (sizeof(C) == 8) {
        const double cs2 = kCS2;
        return kWd[d] * rho * (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    } else {
        return (C)kWd[d] * rho * (C(1) + C(3) * cu + C(4.5) * (cu * cu) - C(1.5) * uu);
    }
}

// f^eq_d(rho, u) - w_d rho_f with rho = rho_f + drho, Eq. (BGKequili) written for the
// deviation from the rest state: w_d (drho + rho (c.u / c_s^2 + (c.u)^2 / (2 c_s^4) - u.u /
// (2 c_s^2)))
template <typename C>
__device__ __forceinline__ C feq_dev(int d, C drho, C rho, C ux, C uy, C uz, C uu)
{
    const C cu = cdot(d, ux, uy, uz);
    if constexpr (sizeof(C) == 8) {
        const double cs2 = kCS2;
        return kWd[d] * (drho + rho * (cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2)));
    } else {
        // FP32 collision arithmetic with fused multiply-adds (uu3 = 1.5 u.u)
        const C uu3 = C(1.5) * uu;
        const C poly = __builtin_fmaf(C(4.5) * cu, cu, __builtin_fmaf(C(3), cu, -uu3));
        return (C)kWd[d] * __builtin_fmaf(rho, poly, drho);
    }
}

// stored value of population d -> deviation f_d - w_d rho_f (FP32 stores the deviation;
// the 16-bit forms store q = f / w_d - rho_f, so the deviation is w_d q)
template <int P>
__device__ __forceinline__ typename Prec<P>::C decode_dev(typename Prec<P>::S v, int d, double rho_f)
{
    using C = typename Prec<P>::C;
    if constexpr (P == PREC_FP64) return v - (C)(kWd[d] * rho_f);
    else if constexpr (P == PREC_FP32) return v;
    else if constexpr (P == PREC_FP16DEV) return (float)kWd[d] * (float)v;
    else return (float)kWd[d] * bf16_to_f32(v);
}

// deviation f_d - w_d rho_f -> stored value of population d
template <int P>
__device__ __forceinline__ void store_dev(typename Prec<P>::S *a, unsigned idx, int d, typename Prec<P>::C df,
                                          double rho_f)
{
    using S = typename Prec<P>::S;
    using C = typename Prec<P>::C;
    if constexpr (P == PREC_FP64) sto(a, idx, (S)((C)(kWd[d] * rho_f) + df));
    else if constexpr (P == PREC_FP32) sto(a, idx, df);
    else if constexpr (P == PREC_FP16DEV) sto(a, idx, (S)(df * kInvW[d]));
    else sto(a, idx, f32_to_bf16(df * kInvW[d]));
}

// Record of one link slot of a fluid node for this step's link pass: the deviation part of
// sum 2 c_d f~_d(x,t) over the slot's links (as G = sum c_d (f~_d - w_d rho_f); the
// rest-state part comes from counts) and the link directions; FP32 float4, FP64 2 x double2,
// at [slot][storage slot of the node]
template <int P>
__device__ __forceinline__ void put_record(const DevSet &s, int g, long long gr, typename Prec<P>::C G0,
                                           typename Prec<P>::C G1, typename Prec<P>::C G2, unsigned grp)
{
    if constexpr (sizeof(typename Prec<P>::C) == 4) {
        reinterpret_cast<float4 *>(s.frec)[g * s.ncell_total + gr] = make_float4(G0, G1, G2, __uint_as_float(grp));
    } else {
        double2 *r = reinterpret_cast<double2 *>(s.frec) + 2 * (g * s.ncell_total + gr);
        r[0] = make_double2(G0, G1);
        r[1] = make_double2(G2, __longlong_as_double((long long)grp));
    }
}
template <int P>
__device__ __forceinline__ unsigned get_record(const DevSet &s, int g, long long gr, double &G0, double &G1, double &G2)
{
    if constexpr (sizeof(typename Prec<P>::C) == 4) {
        const float4 v = reinterpret_cast<const float4 *>(s.frec)[g * s.ncell_total + gr];
        G0 = v.x; G1 = v.y; G2 = v.z;
        return __float_as_uint(v.w);
    } else {
        const double2 *r = reinterpret_cast<const double2 *>(s.frec) + 2 * (g * s.ncell_total + gr);
        const double2 a = r[0], b = r[1];
        G0 = a.x; G1 = a.y; G2 = b.x;
        return (unsigned)__double_as_longlong(b.y);
    }
}

// Rank of a true predicate among the workgroup's threads (thread order) and the total.
__device__ __forceinline__ int block_rank(bool pred, int &total, int *cnt4)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(pred);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) cnt4[wv] = __popcll(bal);
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wv; ++w) off += cnt4[w];
    total = cnt4[0] + cnt4[1] + cnt4[2] + cnt4[3];
    __syncthreads();
    return off + before;
}

// ---------------------------------------------------------------------------
// link words
// ---------------------------------------------------------------------------
__device__ __forceinline__ const MemberDev *member_of_cell(const DevSet &s, long long c)
{
    int lo = 0, hi = s.nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.mem[mid].cell_off <= c) lo = mid;
        else hi = mid - 1;
    }
    return s.mem + lo;
}

// Storage slot of node (i, j, k) under compact storage: its rank among the listed nodes
// of plane k, from the row table of its 32-node word; -1 when the node is not listed.
__device__ __forceinline__ int slot_of(const DevSet &s, const MemberDev *M, int i, int j, int k)
{
    const uint2 r = s.rt[M->rt_off + ((long long)k * M->ny + j) * M->nw + (i >> 5)];
    const unsigned b = 1u << (i & 31);
    return (r.x & b) ? k * (M->nx * M->ny) + (int)r.y + __popc(r.x & (b - 1u)) : -1;
}

// Storage slot of local node `cell` = (i, j, k): the node itself, or its compact slot.
__device__ __forceinline__ int node_slot(const DevSet &s, const MemberDev *M, int cell, int i, int j, int k)
{
    return s.compact ? slot_of(s, M, i, j, k) : cell;
}

template <typename T>
__device__ __forceinline__ void move_values(const char *src, long long from, char *dst, long long to, long long stride)
{
    const T *a = reinterpret_cast<const T *>(src);
    T *b = reinterpret_cast<T *>(dst);
    for (int d = 0; d < kQ; ++d) b[d * stride + to] = a[d * stride + from];
}

// Link words of node (i, j, k) of lattice M from the node map own (this lattice's part):
// for a fluid node x, the directions e whose source x - c_e lies inside a particle and the
// slot (0..3, in the order the particles are met) of the particle owning each source; on
// a narrow lattice a slot is a (particle, image) pair, the image of each source found from
// the particle positions X (the set's array at time t).
__device__ void link_words(const MemberDev *M, const int *own, const double *X, int i, int j, int k,
                           unsigned long long &w0, unsigned long long &w1)
{
    const int nx = M->nx, ny = M->ny, nz = M->nz;
    w0 = 0ull;
    w1 = 0ull;
    if (own[(k * ny + j) * nx + i] >= 0) return;
    unsigned mask = 0u, lo = 0u, hi = 0u;
    int id[4] = {-1, -1, -1, -1}, img[4] = {0, 0, 0, 0};
    int nid = 0;
    bool over = false;
#pragma unroll 1
    for (int e = 0; e < kQ - 1; ++e) {
        int c[3] = {i - kCXd[e], j - kCYd[e], k - kCZd[e]};
        const int u[3] = {c[0], c[1], c[2]};
        const int dims[3] = {nx, ny, nz};
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            if (c[a] < 0 || c[a] >= dims[a]) {
                if (M->per[a]) c[a] = c[a] < 0 ? c[a] + dims[a] : c[a] - dims[a];
                else ok = false;
            }
        }
        if (!ok) continue;
        const int o = own[(c[2] * ny + c[1]) * nx + c[0]];
        if (o < 0) continue;
        const int q = o - M->p_off;
        const int im = source_image(M, u[0], u[1], u[2], X + 3 * (long long)o);
        int sl = 0;
        while (sl < nid && (id[sl] != q || img[sl] != im)) ++sl;
        if (sl == nid) {
            if (nid == 4) { over = true; continue; }
            img[nid] = im;
            id[nid++] = q;
        }
        mask |= 1u << e;
        if (sl & 1) lo |= 1u << e;
        if (sl & 2) hi |= 1u << e;
    }
    if (mask == 0u && !over) return;
    w0 = (unsigned long long)mask | ((unsigned long long)lo << 18) |
         ((unsigned long long)max(id[0], 0) << 36) | ((unsigned long long)max(id[1], 0) << 49) |
         ((unsigned long long)(nid > 2) << 62) | ((unsigned long long)over << 63);
    w1 = (unsigned long long)hi | ((unsigned long long)max(id[2], 0) << 18) | ((unsigned long long)max(id[3], 0) << 31);
}

// Directions of slot g and the slot's local particle index, from the two link words.
__device__ __forceinline__ unsigned slot_dirs(unsigned long long w0, unsigned long long w1, int g, int &id)
{
    const unsigned mask = (unsigned)w0 & 0x3ffffu, lo = (unsigned)(w0 >> 18) & 0x3ffffu;
    const unsigned hi = (unsigned)w1 & 0x3ffffu;
    id = (g == 0) ? (int)(w0 >> 36) & 0x1fff : (g == 1) ? (int)(w0 >> 49) & 0x1fff
       : (g == 2) ? (int)(w1 >> 18) & 0x1fff : (int)(w1 >> 31) & 0x1fff;
    return mask & ((g & 1) ? lo : ~lo) & ((g & 2) ? hi : ~hi);
}

// Compact copy of a listed node's first link word: the word without its overflow bit for
// a fluid node, kSolidWord for a solid one.
constexpr unsigned long long kSolidWord = 1ull << 63;
__device__ __forceinline__ unsigned long long compact_word(unsigned long long w0, bool solid)
{
    return solid ? kSolidWord : (w0 & ~kSolidWord);
}

// Marks the chunks of q's shell list whose z-slab lies within one plane of z.
__device__ __forceinline__ void mark_dirty(const DevSet &s, const MemberDev *M, int q, int z, long long t)
{
    if (q < 0) return;
    const int z0 = s.lzr[2 * q], hz = s.lzr[2 * q + 1];
    if (hz <= 0) return;
    int dz = z - z0;
    if (M->per[2]) dz = ((dz % M->nz) + M->nz) % M->nz;
    for (int w = dz - 1; w <= dz + 1; ++w) {
        const int c = (w >= 0) ? w / hz : -1;
        if (c >= 0 && c < kChunks) s.ldirty[q * kChunks + c] = t;
    }
}

// Link words of a node changed (re-projection of the previous step): the cached link
// entries of every particle named in the old or the new words are stale in the chunks
// around the node's plane z (a particle's slot at the node can move even when its own
// links there do not change).
__device__ __forceinline__ void mark_words(const DevSet &s, const MemberDev *M, unsigned long long o0,
                                           unsigned long long o1, unsigned long long n0, unsigned long long n1,
                                           int z, long long stamp)
{
    for (int g = 0; g < 4; ++g) {
        int q;
        if (slot_dirs(o0, o1, g, q) != 0u) mark_dirty(s, M, M->p_off + q, z, stamp);
        if (slot_dirs(n0, n1, g, q) != 0u) mark_dirty(s, M, M->p_off + q, z, stamp);
    }
}

// ---------------------------------------------------------------------------
// fluid kernel
// ---------------------------------------------------------------------------
// FP32 copy of a particle's wall state for the fluid kernel: X, V, Omega, padding
__device__ __forceinline__ void pack_state(float *o, const double *X, const double *V, const double *W)
{
    for (int a = 0; a < 3; ++a) { o[a] = (float)X[a]; o[4 + a] = (float)V[a]; o[8 + a] = (float)W[a]; }
    o[3] = o[7] = o[11] = 0.0f;
}

__device__ __forceinline__ float mimg_f(float dx, int per, float n)
{
    if (per) {
        if (dx > 0.5f * n) dx -= n;
        else if (dx < -0.5f * n) dx += n;
    }
    return dx;
}

// V_b = V + Omega x r at node (i, j, k) from a packed FP32 state q (X, V, Omega), r the
// node's position relative to the image of the particle that holds link group grp (the
// minimum image, or from a link's midpoint in a set with a narrow lattice, as group_arm)
template <bool NR>
__device__ __forceinline__ void wall_velocity_f(const MemberDev *M, const float4 (&q)[3], unsigned grp, int i, int j,
                                                int k, float &u0, float &u1, float &u2)
{
    float r0, r1, r2;
    if constexpr (NR) {
        const int e = __ffs(grp) - 1;
        const float h0 = 0.5f * (float)kCXd[e], h1 = 0.5f * (float)kCYd[e], h2 = 0.5f * (float)kCZd[e];
        r0 = mimg_f(((float)i - h0) - q[0].x, M->per[0], (float)M->box[0]) + h0;
        r1 = mimg_f(((float)j - h1) - q[0].y, M->per[1], (float)M->box[1]) + h1;
        r2 = mimg_f(((float)k - h2) - q[0].z, M->per[2], (float)M->box[2]) + h2;
    } else {
        r0 = mimg_f((float)i - q[0].x, M->per[0], (float)M->box[0]);
        r1 = mimg_f((float)j - q[0].y, M->per[1], (float)M->box[1]);
        r2 = mimg_f((float)k - q[0].z, M->per[2], (float)M->box[2]);
    }
    u0 = q[1].x + (q[2].y * r2 - q[2].z * r1);
    u1 = q[1].y + (q[2].z * r0 - q[2].x * r2);
    u2 = q[1].z + (q[2].x * r1 - q[2].y * r0);
}

// Velocity of particle q's surface for the links of group grp at node (i, j, k), V_b = V +
// Omega x r with r = x - X (the image that holds the group, as group_arm), in the
// collision precision C; used with c_d . V_b for the link (x, d), which equals c_d . V_b
// at the link's midpoint since c_d . (Omega x c_d) = 0.  X is the position at time t, V
// and Omega the velocities of the step (written by the motion kernel at the other parity).
template <typename C, bool NR>
__device__ __forceinline__ void wall_velocity(const DevSet &s, const MemberDev *M, int q, unsigned grp, int i, int j,
                                              int k, int par, C &u0, C &u1, C &u2)
{
    const double *X = s.X[par] + 3 * q, *V = s.V[par ^ 1] + 3 * q, *W = s.W[par ^ 1] + 3 * q;
    double a0, a1, a2;
    group_arm<NR>(M, grp, i, j, k, X[0], X[1], X[2], a0, a1, a2);
    const C r0 = (C)a0, r1 = (C)a1, r2 = (C)a2;
    const C w0 = (C)W[0], w1 = (C)W[1], w2 = (C)W[2];
    u0 = (C)V[0] + (w1 * r2 - w2 * r1);
    u1 = (C)V[1] + (w2 * r0 - w0 * r2);
    u2 = (C)V[2] + (w0 * r1 - w1 * r0);
}

// Wall velocity of particle q for the link group grp at node (i, j, k), from the packed
// FP32 state (FP32 and 16-bit storage) or the FP64 state.
template <typename C, bool NR>
__device__ __forceinline__ void slot_velocity(const DevSet &s, const MemberDev *M, int q, unsigned grp, int i, int j,
                                              int k, int par, C &u0, C &u1, C &u2)
{
    if constexpr (sizeof(C) == 4) {
        const float4 *pq = reinterpret_cast<const float4 *>(s.pf[par] + 12 * (M->p_off + q));
        const float4 qq[3] = {pq[0], pq[1], pq[2]};
        wall_velocity_f<NR>(M, qq, grp, i, j, k, u0, u1, u2);
    } else {
        wall_velocity<C, NR>(s, M, M->p_off + q, grp, i, j, k, par, u0, u1, u2);
    }
}

// Eq. (mem) for the links of a fluid node: f_e = f~_d(x,t) - 2 (w_d / c_s^2) rho_f V_b . c_d,
// d = e*, for every direction e whose source is inside a particle; f[e] holds the deviation
// f~_d(x,t) - w_d rho_f (the same relation holds for deviations since w_e = w_d).  V_b comes
// from the particle's position at t and its velocities of the step; the momentum these
// links exchange was accounted for by the link pass and the motion kernel.
template <typename C, bool NR>
__device__ __forceinline__ void moving_wall(const DevSet &s, const MemberDev *M, C (&f)[kQ], unsigned long long w0,
                                            int i, int j, int k, int par, double rho_f, long long gc)
{
    const unsigned mask = (unsigned)w0 & 0x3ffffu, lo = (unsigned)(w0 >> 18) & 0x3ffffu;
    const unsigned long long w1 = (w0 >> 62) ? s.lw[s.ncell_total + gc] : 0ull;
    const unsigned hi = (unsigned)w1 & 0x3ffffu;
    // slots 0 and 1 together: both particle states are loaded at once, then every direction
    // takes the velocity of its slot without a branch
    const unsigned g0 = mask & ~lo & ~hi, g1 = mask & lo & ~hi;
    C a0, a1, a2, b0, b1, b2;
    slot_velocity<C, NR>(s, M, (int)(w0 >> 36) & 0x1fff, g0 ? g0 : 1u, i, j, k, par, a0, a1, a2);
    slot_velocity<C, NR>(s, M, (int)(w0 >> 49) & 0x1fff, g1 ? g1 : 1u, i, j, k, par, b0, b1, b2);
#pragma unroll
    for (int e = 0; e < kQ - 1; ++e) {
        const int d = kOPP[e];
        const bool one = (lo >> e) & 1u;
        const C u0 = one ? b0 : a0, u1 = one ? b1 : a1, u2 = one ? b2 : a2;
        const C cu = cdot(d, u0, u1, u2);
        const C m = (((mask & ~hi) >> e) & 1u) ? (C)(kMW[d] * rho_f) : C(0);
        f[e] = f[e] - m * cu;
    }
    // slots 2 and 3 (nodes bordering more than two particles)
    if (hi != 0u) {
#pragma unroll 1
        for (int g = 2; g < 4; ++g) {
            int q;
            const unsigned grp = slot_dirs(w0, w1, g, q);
            if (grp == 0u) continue;
            C u0, u1, u2;
            slot_velocity<C, NR>(s, M, q, grp, i, j, k, par, u0, u1, u2);
#pragma unroll
            for (int e = 0; e < kQ - 1; ++e) {
                const int d = kOPP[e];
                const C cu = cdot(d, u0, u1, u2);
                const C m = ((grp >> e) & 1u) ? (C)(kMW[d] * rho_f) : C(0);
                f[e] = f[e] - m * cu;
            }
        }
    }
}

// Start of step t: brings the other node map up to date with the re-projection of step
// t-1 (its change list, or a full copy after an overflow or a particle set-up), refreshes
// the link words of the changed nodes and their neighbours (all of them after a full
// copy) from the node map of step t, and opens the change list of step t.
template <int P>
__global__ __launch_bounds__(256) void k_refresh(DevSet s)
{
    using S = typename Prec<P>::S;
    const long long t = *s.tstep;
    // (both change counts and the list-rebuild step are loaded with the step counter)
    const int cnt0 = s.chgcnt[0], cnt1 = s.chgcnt[1];
    const long long relist_at = *s.relist_at;
    const int par = (int)(t & 1);
    const int cnt = par ? cnt0 : cnt1;
    const bool relist = s.listmode && relist_at == t;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool over = false;
    // (a step that rebuilds the node lists rewrites every compact word in the record kernel)
    const bool fix_compact = s.compact && !relist;
    if (cnt > s.chg_cap) {
        // (every link word may change: the record kernel rewrites every compact word)
        if (t0 == 0) *s.lwc_bad = t;
        for (long long c = t0; c < s.ncell_total; c += stride) {
            s.own[par ^ 1][c] = s.own[par][c];
            const MemberDev *M = member_of_cell(s, c);
            const int cell = (int)(c - M->cell_off);
            const int nxy = M->nx * M->ny;
            const int k = cell / nxy, rem = cell - k * nxy, j = rem / M->nx, i = rem - j * M->nx;
            unsigned long long w0, w1;
            link_words(M, s.own[par] + M->cell_off, s.X[par], i, j, k, w0, w1);
            const unsigned long long o0 = s.lw[c], o1 = s.lw[s.ncell_total + c];
            if (o0 != w0 || o1 != w1) mark_words(s, M, o0, o1, w0, w1, k, t - 1);
            s.lw[c] = w0;
            s.lw[s.ncell_total + c] = w1;
            over |= (w0 >> 63) != 0ull;
        }
    } else {
        const int *lst = s.chg[par ^ 1];
        for (long long e = t0; e < cnt; e += stride) s.own[par ^ 1][lst[2 * e]] = lst[2 * e + 1];
        // the words of the changed nodes and their neighbours: one group of 32 lanes per
        // word, lane e < 18 reading the owner of source e and lane 18 the node's own (one
        // round of loads), every lane assembling the word from the group's values as
        // link_words does, lane 0 storing it
        const int lane = threadIdx.x & 31;
        const long long grp = t0 >> 5, ngrp = stride >> 5;
        for (long long w = grp; w < (long long)cnt * kQ; w += ngrp) {
            const long long ch = w / kQ;
            const int q = (int)(w - ch * kQ); // 18: the changed node itself
            const long long gcell = lst[2 * ch];
            const MemberDev *M = member_of_cell(s, gcell);
            const int nx = M->nx, ny = M->ny, nz = M->nz;
            const int c0 = (int)(gcell - M->cell_off);
            const int k0 = c0 / (nx * ny), rem = c0 - k0 * nx * ny, j0 = rem / nx, i0 = rem - j0 * nx;
            // a neighbour across a bounded face wraps to a node whose words are unchanged;
            // recomputing them is harmless
            const int ci = wrapc(i0 + kCXd[q], nx), cj = wrapc(j0 + kCYd[q], ny), ck = wrapc(k0 + kCZd[q], nz);
            const int *own = s.own[par] + M->cell_off;
            // the node's current words, loaded with the owners (lane 0 compares and stores)
            const long long gc = M->cell_off + (ck * ny + cj) * nx + ci;
            unsigned long long o0 = 0ull, o1 = 0ull;
            if (lane == 0) { o0 = s.lw[gc]; o1 = s.lw[s.ncell_total + gc]; }
            int o = -1, im = 0;
            if (lane < kQ - 1) {
                const int si = ci - kCXd[lane], sj = cj - kCYd[lane], sk = ck - kCZd[lane];
                const bool ok = (M->per[0] || (si >= 0 && si < nx)) && (M->per[1] || (sj >= 0 && sj < ny)) &&
                                (M->per[2] || (sk >= 0 && sk < nz));
                if (ok) o = own[(wrapc(sk, nz) * ny + wrapc(sj, ny)) * nx + wrapc(si, nx)];
                if (o >= 0) im = source_image(M, si, sj, sk, s.X[par] + 3 * (long long)o);
            } else if (lane == kQ - 1) {
                o = own[(ck * ny + cj) * nx + ci];
            }
            const int self = __shfl(o, kQ - 1, 32);
            unsigned mask = 0u, slo = 0u, shi = 0u;
            int id0 = -1, id1 = -1, id2 = -1, id3 = -1;
            bool ov = false;
            if (self < 0) {
                // (on a narrow lattice a slot is a (particle, image) pair: the key packs both)
                for (int e = 0; e < kQ - 1; ++e) {
                    const int oe = __shfl(o, e, 32);
                    if (oe < 0) continue;
                    const int pq = (oe - M->p_off) | (__shfl(im, e, 32) << 24);
                    int sl;
                    if (id0 < 0 || id0 == pq) { id0 = pq; sl = 0; }
                    else if (id1 < 0 || id1 == pq) { id1 = pq; sl = 1; }
                    else if (id2 < 0 || id2 == pq) { id2 = pq; sl = 2; }
                    else if (id3 < 0 || id3 == pq) { id3 = pq; sl = 3; }
                    else { ov = true; continue; }
                    mask |= 1u << e;
                    if (sl & 1) slo |= 1u << e;
                    if (sl & 2) shi |= 1u << e;
                }
            }
            unsigned long long w0 = 0ull, w1 = 0ull;
            if (mask != 0u || ov) {
                w0 = (unsigned long long)mask | ((unsigned long long)slo << 18) |
                     ((unsigned long long)(max(id0, 0) & 0x1fff) << 36) |
                     ((unsigned long long)(max(id1, 0) & 0x1fff) << 49) |
                     ((unsigned long long)(id2 >= 0) << 62) | ((unsigned long long)ov << 63);
                w1 = (unsigned long long)shi | ((unsigned long long)(max(id2, 0) & 0x1fff) << 18) |
                     ((unsigned long long)(max(id3, 0) & 0x1fff) << 31);
            }
            // a changed word marks the chunks around plane ck of every particle it names,
            // old or new: lane l < 8 takes slot l & 3 of the old (l < 4) or the new words, so
            // the particles' chunk layouts are loaded in one round
            const unsigned long long g0w = __shfl(o0, 0, 32), g1w = __shfl(o1, 0, 32);
            if ((g0w != w0 || g1w != w1) && lane < 8) {
                int q;
                const unsigned dirs = (lane < 4) ? slot_dirs(g0w, g1w, lane & 3, q) : slot_dirs(w0, w1, lane & 3, q);
                if (dirs != 0u) mark_dirty(s, M, M->p_off + q, ck, t - 1);
            }
            // the node's compact word at its storage slot, when listed
            const int ns = fix_compact ? node_slot(s, M, (ck * ny + cj) * nx + ci, ci, cj, ck) : -1;
            if (lane == 0) {
                s.lw[gc] = w0;
                s.lw[s.ncell_total + gc] = w1;
                if (ns >= 0) s.lwc[M->cell_off + ns] = compact_word(w0, self >= 0);
                over |= ov;
            }
        }
    }
    if (over) atomicOr(s.flags, 0x80u);

    // node lists, when a particle has moved the skin since they were built (or after a
    // set-up): per z plane, in x-fastest order, every fluid node and every solid node
    // less than the skin inside its particle's surface.  Only such a node can become
    // fluid before a particle has moved the skin.  The skin follows the lattice's
    // fastest particle (kSkinSteps of its last step, within [kSkinMin, kListSkin]).
    if (relist) {
        __shared__ int cnt4[4];
        __shared__ double vred[4];
        for (long long q = t0; q < s.ptot; q += stride)
            for (int ax = 0; ax < 3; ++ax) s.Xl[3 * q + ax] = s.X[par][3 * q + ax];
        for (int pl = blockIdx.x; pl < s.nplanes; pl += gridDim.x) {
            int lo = 0, hi = s.nmem - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s.mem[mid].pz_off <= pl) lo = mid;
                else hi = mid - 1;
            }
            const MemberDev *M = s.mem + lo;
            const int z = pl - M->pz_off, nx = M->nx, nxy = M->nx * M->ny;
            const int *own = s.own[par] + M->cell_off;
            int *lst = s.clist + M->cell_off + (long long)z * nxy;
            // the lattice's largest particle step (non-negative: bit patterns order)
            double vm = 0.0;
            for (int q = threadIdx.x; q < M->np; q += blockDim.x) vm = fmax(vm, s.pspd[M->p_off + q]);
            for (int off = 32; off >= 1; off >>= 1) vm = fmax(vm, __shfl_xor(vm, off, 64));
            __syncthreads();
            if ((threadIdx.x & 63) == 0) vred[threadIdx.x >> 6] = vm;
            __syncthreads();
            vm = fmax(fmax(vred[0], vred[1]), fmax(vred[2], vred[3]));
            const double skin = fmin(fmax(kSkinSteps * vm, kSkinMin), kListSkin);
            if (threadIdx.x == 0) s.skin[lo] = skin;
            const int oldcnt = s.ccnt[pl];
            int count = 0;
            int chg = 0; // the plane's list differs from the previous one
            for (int c0 = 0; c0 < nxy; c0 += blockDim.x) {
                const int c = c0 + threadIdx.x;
                bool listed = false;
                int cell = 0;
                if (c < nxy) {
                    cell = z * nxy + c;
                    const int o = own[cell];
                    if (o < 0) {
                        listed = true;
                    } else {
                        const double rr = s.R[o] - skin;
                        const int j = c / nx, i = c - j * nx;
                        const double *Xq = s.X[par] + 3 * o;
                        listed = rr <= 0.0 || dist2(M, i, j, z, Xq[0], Xq[1], Xq[2]) > rr * rr;
                    }
                }
                int tot = 0;
                const int rk = block_rank(listed, tot, cnt4);
                if (listed) {
                    chg |= (count + rk >= oldcnt || lst[count + rk] != cell) ? 1 : 0;
                    lst[count + rk] = cell;
                }
                count += tot;
            }
            // compact storage: an unchanged list keeps its slots, nothing moves
            const bool moved = __syncthreads_or(chg) || count != oldcnt;
            if (threadIdx.x == 0) s.ccnt[pl] = count;
            if (s.compact && moved) {
                // compact storage: move the plane's populations to the new list order
                // (through the scratch buffer), then rewrite the plane's row tables
                __shared__ unsigned tab[kMaxPlaneWords];
                __threadfence_block();
                __syncthreads();
                const long long nc = M->ncell, po = M->pop_off * (long long)s.es;
                char *A = (char *)(par ? s.popB : s.popA) + po;
                char *Cb = (char *)s.popC + po;
                const int ny = M->ny, nw = M->nw;
                for (int k = threadIdx.x; k < count; k += blockDim.x) {
                    const int c = lst[k] - z * nxy, j = c / nx, i = c - j * nx;
                    const int old = slot_of(s, M, i, j, z);
                    const long long to = (long long)z * nxy + k;
                    if (old < 0) {
                        // not listed before: a node uncovered in the last re-projection
                        // takes its parked refill f^eq(rho_bar, V_b) (Eq. convertSF); any
                        // other is solid and takes the rest state w_d rho_f until refilled
                        const long long gcell = M->cell_off + lst[k];
                        const int pi = s.pend[gcell];
                        double rb = M->rho_f, u0 = 0.0, u1 = 0.0, u2 = 0.0;
                        if (pi >= 0) {
                            const double *rec = s.pbuf[par ^ 1] + 4 * pi;
                            rb = rec[0]; u0 = rec[1]; u1 = rec[2]; u2 = rec[3];
                            s.pend[gcell] = -1;
                        }
                        const double uu = u0 * u0 + u1 * u1 + u2 * u2;
                        S *CbS = reinterpret_cast<S *>(Cb);
                        for (int d = 0; d < kQ; ++d)
                            st<P>(CbS, (unsigned)(d * nc + to), d, (typename Prec<P>::C)feq<double>(d, rb, u0, u1, u2, uu),
                                  M->rho_f);
                        continue;
                    }
                    if (s.es == 8) move_values<unsigned long long>(A, old, Cb, to, nc);
                    else if (s.es == 4) move_values<unsigned>(A, old, Cb, to, nc);
                    else move_values<unsigned short>(A, old, Cb, to, nc);
                }
                for (int w = threadIdx.x; w < ny * nw; w += blockDim.x) tab[w] = 0u;
                __threadfence_block();
                __syncthreads();
                for (int k = threadIdx.x; k < count; k += blockDim.x) {
                    const int c = lst[k] - z * nxy, j = c / nx, i = c - j * nx;
                    atomicOr(&tab[j * nw + (i >> 5)], 1u << (i & 31));
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    unsigned run = 0u;
                    uint2 *rtp = s.rt + M->rt_off + (long long)z * ny * nw;
                    for (int w = 0; w < ny * nw; ++w) {
                        rtp[w] = make_uint2(tab[w], run);
                        run += __popc(tab[w]);
                    }
                }
                for (int k = threadIdx.x; k < count; k += blockDim.x) {
                    const long long at = (long long)z * nxy + k;
                    if (s.es == 8) move_values<unsigned long long>(Cb, at, A, at, nc);
                    else if (s.es == 4) move_values<unsigned>(Cb, at, A, at, nc);
                    else move_values<unsigned short>(Cb, at, A, at, nc);
                }
                __threadfence_block();
                __syncthreads();
            }
        }
    }
    if (t0 == 0) {
        s.chgcnt[par] = 0;
        s.pcnt[par] = 0; // parked refills of this step's re-projection
        *s.tcopy = t; // the re-projection kernel of this step reads the step from here
    }
}

template <bool NR>
__device__ __forceinline__ void rebuild_chunk(const DevSet &s, int p, int chunk, long long t, int *lc, unsigned *lg);
constexpr int kLinkLds = 384; // entries of a rebuilt chunk kept in LDS for its link-set sums

// Workgroups of the record kernel that rebuild stale link chunks, four chunks each.
__host__ __device__ __forceinline__ int rebuild_blocks(const DevSet &s) { return (s.ptot * kChunks + 3) / 4; }

// After the refresh (link words and storage slots of step t final): first the rebuild of
// the stale link chunks (rebuild_chunk), one wave per (particle, chunk); then the link
// records of step t for the link pass, one thread per listed node (or per node of a dense
// tile) on the fluid kernel's grid: per fluid node with links and per slot of its link
// words, G = sum c_d (f~_d(x,t) - w_d rho_f) over the slot's links, read from the node's
// own storage slot (consecutive threads read consecutive slots).
template <int P, bool CMP, bool NR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == PREC_FP64 ? 4 : 6))) void k_records(DevSet s)
{
    using S = typename Prec<P>::S;
    using C = typename Prec<P>::C;
    const long long t = *s.tstep;
    const int par = (int)(t & 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) *s.rec_step = t;
    // the first workgroups rebuild the stale link chunks, one wave per chunk: those waves
    // are few, long and latency-bound, so they start first and run beside the node waves
    const int nrb = rebuild_blocks(s);
    if ((int)blockIdx.x < nrb) {
        __shared__ int rb_c[4][kLinkLds];
        __shared__ unsigned rb_g[4][kLinkLds];
        const int wv = (int)(threadIdx.x >> 6);
        const int ci = (int)blockIdx.x * 4 + wv;
        if (ci < s.ptot * kChunks) rebuild_chunk<NR>(s, ci / kChunks, ci - (ci / kChunks) * kChunks, t, rb_c[wv], rb_g[wv]);
        return;
    }
    const int g = xcd_swizzle((int)blockIdx.x - nrb, (int)gridDim.x - nrb);
    const MemberDev *M = member_of_tile(s, g);
    const int tl = g - uni(M->tile_off);
    const int ntx = uni(M->ntx), nty = uni(M->nty);
    const int nx = uni(M->nx), ny = uni(M->ny), nz = uni(M->nz);
    const int nxy = nx * ny;
    const unsigned nc = (unsigned)uni(M->ncell);
    const long long cell_off = uni(M->cell_off);
    const S *A = (const S *)(par ? s.popB : s.popA) + uni(M->pop_off);
    const double rho_f = uni(M->rho_f);
    // compact storage: every listed node's compact word is rewritten here after a list
    // rebuild or a full copy of the node map, and read from its slot otherwise
    const bool full_compact = CMP && (*s.relist_at == t || *s.lwc_bad == t);
    const int *own = s.own[par] + cell_off;
    auto records = [&](int cell, int slot) {
        const long long gc = cell_off + cell;
        unsigned long long w0;
        if constexpr (CMP) {
            if (full_compact) {
                w0 = compact_word(s.lw[gc], own[cell] >= 0);
                s.lwc[cell_off + slot] = w0;
            } else {
                w0 = s.lwc[cell_off + slot];
            }
            if (w0 & kSolidWord) return;
        } else {
            w0 = s.lw[gc];
        }
        if (((unsigned)w0 & 0x3ffffu) == 0u) return;
        const unsigned long long w1 = (w0 >> 62) ? s.lw[s.ncell_total + gc] : 0ull;
        const int ng = (w0 >> 62) ? 4 : 2;
        // the node's populations in the link directions, loaded without a branch
        const unsigned all = (unsigned)w0 & 0x3ffffu;
        C v[kQ - 1];
#pragma unroll
        for (int e = 0; e < kQ - 1; ++e) {
            const int d = kOPP[e];
            const bool on = (all >> e) & 1u;
            // (every lane loads; a lane without the link reads the array's first element)
            const C x = decode_dev<P>(ldo(A, on ? (unsigned)d * nc + (unsigned)slot : 0u), d, rho_f);
            v[e] = on ? x : C(0);
        }
        // slots 0 and 1 in one pass without branches (v is 0 outside the links)
        const unsigned lo = (unsigned)(w0 >> 18) & 0x3ffffu, hi = (unsigned)w1 & 0x3ffffu;
        const unsigned g0 = all & ~lo & ~hi, g1 = all & lo & ~hi;
        C A0 = C(0), A1 = C(0), A2 = C(0), B0 = C(0), B1 = C(0), B2 = C(0);
#pragma unroll
        for (int e = 0; e < kQ - 1; ++e) {
            const int d = kOPP[e];
            const C va = ((g0 >> e) & 1u) ? v[e] : C(0), vb = ((g1 >> e) & 1u) ? v[e] : C(0);
            if (kCX[d] > 0) { A0 += va; B0 += vb; } else if (kCX[d] < 0) { A0 -= va; B0 -= vb; }
            if (kCY[d] > 0) { A1 += va; B1 += vb; } else if (kCY[d] < 0) { A1 -= va; B1 -= vb; }
            if (kCZ[d] > 0) { A2 += va; B2 += vb; } else if (kCZ[d] < 0) { A2 -= va; B2 -= vb; }
        }
        if (g0 != 0u) put_record<P>(s, 0, cell_off + slot, A0, A1, A2, g0);
        if (g1 != 0u) put_record<P>(s, 1, cell_off + slot, B0, B1, B2, g1);
#pragma unroll 1
        for (int gg = 2; gg < ng; ++gg) {
            int q;
            const unsigned grp = slot_dirs(w0, w1, gg, q);
            if (grp == 0u) continue;
            C G0 = C(0), G1 = C(0), G2 = C(0);
#pragma unroll
            for (int e = 0; e < kQ - 1; ++e) {
                if (!((grp >> e) & 1u)) continue;
                const int d = kOPP[e];
                if (kCX[d] > 0) G0 += v[e]; else if (kCX[d] < 0) G0 -= v[e];
                if (kCY[d] > 0) G1 += v[e]; else if (kCY[d] < 0) G1 -= v[e];
                if (kCZ[d] > 0) G2 += v[e]; else if (kCZ[d] < 0) G2 -= v[e];
            }
            put_record<P>(s, gg, cell_off + slot, G0, G1, G2, grp);
        }
    };
    if (s.listmode) {
        const int lb = tl % ntx, z = tl / ntx;
        const int cnt = s.ccnt[uni(M->pz_off) + z];
        for (int lbx = lb; lbx * 256 < cnt; lbx += ntx) {
            const int kk = lbx * 256 + (int)threadIdx.x;
            if (kk >= cnt) break;
            const int c = s.clist[cell_off + (long long)z * nxy + kk];
            records(c, CMP ? z * nxy + kk : c);
        }
    } else {
        const int bxl = uni(M->bx_log2);
        const int lx = threadIdx.x & ((1 << bxl) - 1), ly = threadIdx.x >> bxl;
        const int tx = tl % ntx, trem = tl / ntx, ty = trem % nty, tz = trem / nty;
        const int i = (tx << bxl) + lx, j = ty * uni(M->by) + ly;
        if (i >= nx || j >= ny) return;
        const int z0 = tz * s.nzt, z1 = min(z0 + s.nzt, nz);
        for (int z = z0; z < z1; ++z) {
            const int c = (z * ny + j) * nx + i;
            records(c, c);
        }
    }
}

// Pull streaming (Eq. stream), stationary half-way walls, moving half-way walls on the
// particles (Eq. mem, from the node's link words), the density faces (Sec. 2.4), BGK
// collision (Eqs. bgk, BGKequili, rhoAndU) and probe partial sums.
template <int P, bool CMP, bool NR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == PREC_FP64 ? 3 : (CMP ? 6 : 5)))) void k_fluid(DevSet s)
{
    using S = typename Prec<P>::S;
    using C = typename Prec<P>::C;
    __shared__ double red[4][8];

    const long long t = *s.tstep;
    const int par = (int)(t & 1);

    const int g = xcd_swizzle(blockIdx.x, gridDim.x);
    const MemberDev *M = member_of_tile(s, g);
    const int tl = g - uni(M->tile_off);
    const int ntx = uni(M->ntx), nty = uni(M->nty);
    const int nx = uni(M->nx), ny = uni(M->ny), nz = uni(M->nz);
    const int nc = (int)uni(M->ncell);
    const int nxy = nx * ny;
    const long long pop_off = uni(M->pop_off), cell_off = uni(M->cell_off);
    const int pz_off = uni(M->pz_off);
    const S *A = (const S *)(par ? s.popB : s.popA) + pop_off;
    S *B = (S *)(par ? s.popA : s.popB) + pop_off;
    const int *own = s.own[par] + cell_off;
    const double rho_fd = uni(M->rho_f);
    const C omega = (C)uni(M->omega);
    const int bc4 = uni(M->bc[4]), bc5 = uni(M->bc[5]);
    // (the rest of the lattice's constants are read here too: the barriers of the node
    // loop below would otherwise make each wave read them again after them)
    const int bc0 = uni(M->bc[0]), bc1 = uni(M->bc[1]), bc2 = uni(M->bc[2]), bc3 = uni(M->bc[3]);
    const long long rt_off = CMP ? uni(M->rt_off) : 0ll;
    const int nw = CMP ? uni(M->nw) : 0, per_x = uni(M->per[0]);
    const long long t_n = uni(M->t_n);
    long long ti = t + 1;
    if (ti > t_n + 1) ti = t_n + 1;
    const C drho_in = (C)(s.wave[uni(M->wave_off) + ti] - rho_fd);

    // CMP: compact storage (node lists, populations at the nodes' ranks in the lists)
    const bool lists = CMP || s.listmode != 0;
    constexpr bool compact = CMP;

    // one chunk of the work: the nodes (i, j) of planes z0 .. z1-1 (dense tiles), or one
    // listed node of plane z0 at slot me0 (node lists); accum adds the probe partial sums
    // to those of an earlier chunk of the same workgroup
    // compact storage: the row-table words of the workgroup's source rows, staged in LDS
    // (rows j0 - 1 .. j1 + 1 of planes z - 1, z, z + 1 for the chunk's nodes in rows j0 .. j1)
    __shared__ uint2 rt_lds[kRtLds];
    __shared__ int jr[2];

    auto run = [&](int i, int j, int z0, int z1, int me0, bool vij, bool accum, const uint2 *lrt, int jb,
                   int nrows, unsigned long long wcl) {
        // offsets to the x-1 / x+1 / y-1 / y+1 neighbours (wrapped on periodic axes) and the
        // kind of face crossed to reach them (0 inside or periodic, 1 wall, 2 density face)
        int oxm = (i > 0) ? -1 : (nx - 1), oxp = (i < nx - 1) ? 1 : -(nx - 1);
        int kxm = (i > 0) ? 0 : bc0, kxp = (i < nx - 1) ? 0 : bc1;
        int oym = (j > 0) ? -nx : (ny - 1) * nx, oyp = (j < ny - 1) ? nx : -(ny - 1) * nx;
        int kym = (j > 0) ? 0 : bc2, kyp = (j < ny - 1) ? 0 : bc3;

        for (int z = z0; z < z1; ++z) {
            // keep the 18 per-direction offsets from being hoisted out of the loop: they are
            // cheap to recompute and would otherwise stay live in 36 registers
            asm volatile("" : "+v"(oxm), "+v"(oxp), "+v"(oym), "+v"(oyp), "+v"(kxm), "+v"(kxp), "+v"(kym), "+v"(kyp));
            const int cell = (z * ny + j) * nx + i;
            bool fl = false;
            unsigned long long wc = 0ull;
            if constexpr (CMP) {
                // the node's compact word, at its slot (loaded with the node's cell)
                wc = wcl;
                fl = vij && !(wc & kSolidWord);
            } else {
                if (vij) fl = ldo(own, (unsigned)cell) < 0;
            }
            double pr0 = 0.0, pr1 = 0.0, pr2 = 0.0, pr3 = 0.0;
            // Dense tiles with 4- and 8-byte storage write every node of a row, so each store
            // covers whole cache lines: a solid node loads nothing and stores the rest state
            // w_d, a value that is never read (a node is refilled on uncovering).  16-bit
            // storage measured faster with solid nodes left out; with node lists only the
            // fluid nodes work.
            constexpr bool kWholeRows = sizeof(S) >= 4;
            if ((kWholeRows && !lists) ? vij : fl) {
                const int ozm = (z > 0) ? -nxy : (nz - 1) * nxy, ozp = (z < nz - 1) ? nxy : -(nz - 1) * nxy;
                const int kzm = (z > 0) ? 0 : bc4, kzp = (z < nz - 1) ? 0 : bc5;
                // Loads are issued for every lane, a solid lane reading the first element of the
                // array (one shared line) instead of branching around each load.
                unsigned long long lwv;
                if constexpr (CMP) {
                    lwv = fl ? wc : 0ull;
                } else {
                    const unsigned long long lwr = s.lw[fl ? cell_off + cell : 0];
                    lwv = fl ? lwr : 0ull;
                }
                const unsigned lmask = (unsigned)lwv & 0x3ffffu;
                // storage slot of this node: the node itself, or its rank in the plane's list
                // (as an offset from the node that the compiler cannot see through: it keeps
                // the register allocation of the node-layout kernel, which has no spills)
                int dlt = compact ? me0 - cell : 0;
                if (compact) asm volatile("" : "+v"(dlt));
                const int me = cell + dlt;
                // compact storage: slots of the sources from the row tables of the 9 source rows
                // (y - c_y, z - c_z).  Along a row the listed nodes hold consecutive slots, so
                // the source x - 1 sits one slot below the node's rank in that row and x + 1
                // one above it (plus one when x itself is listed); a source across a periodic
                // x face reads the table word at the other end of the row.
                int src[kQ - 1];
                if (compact) {
                    const uint2 *rtab = s.rt + rt_off;
                    const unsigned b = 1u << (i & 31);
                    const int wx = (i == 0) ? nx - 1 : 0;
                    const unsigned bw = 1u << (wx & 31);
                    uint2 wv[9], ww[9];
                    if (lrt) {
    #pragma unroll
                        for (int r = 0; r < 9; ++r) {
                            const int row = ((r % 3) * nrows + (j + r / 3 - 1 - jb)) * nw;
                            wv[r] = lrt[row + (i >> 5)];
                            ww[r] = per_x ? lrt[row + (wx >> 5)] : make_uint2(0u, 0u);
                        }
                    } else {
    #pragma unroll
                        for (int r = 0; r < 9; ++r) {
                            const int jj = wrapc(j + r / 3 - 1, ny), zz = wrapc(z + r % 3 - 1, nz);
                            const long long row = ((long long)zz * ny + jj) * nw;
                            wv[r] = rtab[row + (i >> 5)];
                            ww[r] = per_x ? rtab[row + (wx >> 5)] : make_uint2(0u, 0u);
                        }
                    }
    #pragma unroll
                    for (int e = 0; e < kQ - 1; ++e) {
                        const int r = (1 - kCY[e]) * 3 + (1 - kCZ[e]);
                        const int zb = wrapc(z - kCZ[e], nz) * nxy;
                        const int rk = zb + (int)wv[r].y + __popc(wv[r].x & (b - 1u));
                        const int rwr = zb + (int)ww[r].y + __popc(ww[r].x & (bw - 1u));
                        int v;
                        if (kCX[e] == 0) v = rk;
                        else if (kCX[e] < 0) v = (i < nx - 1) ? rk + ((wv[r].x & b) ? 1 : 0) : rwr;
                        else v = (i > 0) ? rk - 1 : rwr;
                        src[e] = max(v, 0);
                    }
                }
                C f[kQ];
                S raw[kQ];
                unsigned unk = 0u;
    #pragma unroll
                for (int e = 0; e < kQ - 1; ++e) {
                    int off = 0, kind = 0;
                    if (kCX[e] > 0) { off += oxm; kind = max(kind, kxm); } else if (kCX[e] < 0) { off += oxp; kind = max(kind, kxp); }
                    if (kCY[e] > 0) { off += oym; kind = max(kind, kym); } else if (kCY[e] < 0) { off += oyp; kind = max(kind, kyp); }
                    if (kCZ[e] > 0) { off += ozm; kind = max(kind, kzm); } else if (kCZ[e] < 0) { off += ozp; kind = max(kind, kzp); }
                    // f_e(x, t+1) = f~_e(x - c_e, t); from a wall or a particle the population
                    // comes back from this node, f~_{e*}(x, t); across a density face it is unknown
                    const bool back = (kind != 0) || ((lmask >> e) & 1u);
                    // (offsets from array e: the select is taken between per-lane offsets, so
                    // that no per-lane multiply by nc is formed)
                    const unsigned from = compact ? (unsigned)src[e] : (unsigned)(cell + off);
                    const unsigned idx = (unsigned)(e * nc) +
                                         (back ? (unsigned)((kOPP[e] - e) * nc) + (unsigned)me : from);
                    raw[e] = ldo(A, fl ? idx : 0u);
                    unk |= (kind == BC_PRESSURE) ? (1u << e) : 0u;
                }
                raw[18] = ldo(A, fl ? (unsigned)(18 * nc) + (unsigned)me : 0u);
                // the arithmetic works on deviations f_d - w_d rho_f from the rest state: Eqs.
                // (stream), (mem) and the density faces are affine with the same coefficients
                // for f and its deviation (w_d = w_{d*}; the weights of each Zou-He closure sum
                // to one), and the deviations keep the small density and momentum signals
                // clear of the rounding of the O(1) rest populations
    #pragma unroll
                for (int e = 0; e < kQ; ++e)
                    f[e] = (fl && !((unk >> e) & 1u)) ? decode_dev<P>(raw[e], e, rho_fd) : C(0);
                if (lmask != 0u) moving_wall<C, NR>(s, M, f, lwv, i, j, z, par, rho_fd, cell_off + cell);

                if (z == 0 && bc4 == BC_PRESSURE) zou_he<C>(f, drho_in, false);
                if (z == nz - 1 && bc5 == BC_PRESSURE) zou_he<C>(f, C(0), true);

                C drho, jx, jy, jz;
                moments<C>(f, drho, jx, jy, jz);
                const C rho = (C)rho_fd + drho;
                // watchdog: a fluid node whose density is not a positive finite number
                // (status 0x400; NaN fails the first comparison)
                if (fl && !(rho > C(0) && rho < C(1e30))) atomicOr(s.flags, 0x400u);
                if (fl) {
                    pr0 = 1.0;
                    pr1 = (double)drho;
                    pr2 = (double)jz;
                    pr3 = rho_fd + (double)drho;
                }
                C ux, uy, uz, uu;
                if constexpr (sizeof(C) == 8) {
                    ux = jx / rho; uy = jy / rho; uz = jz / rho;
                    uu = ux * ux + uy * uy + uz * uz;
                } else {
                    const C ir = C(1) / rho;
                    ux = jx * ir; uy = jy * ir; uz = jz * ir;
                    uu = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
                }
    #pragma unroll
                for (int d = 0; d < kQ; ++d) {
                    const C fe = feq_dev<C>(d, drho, rho, ux, uy, uz, uu);
                    C post;
                    if constexpr (sizeof(C) == 8) post = f[d] + omega * (fe - f[d]);
                    else post = __builtin_fmaf(omega, fe - f[d], f[d]);
                    store_dev<P>(B, (unsigned)(d * nc) + (unsigned)me, d, post, rho_fd);
                }
            }
            const int pidx = s.pzmap[pz_off + z];
            if (pidx >= 0) {
                double v[4] = {pr0, pr1, pr2, pr3};
                block_sum<4>(v, red);
                if (threadIdx.x == 0) {
                    double *o = s.pprt + ((long long)g * s.nzt + (z - z0)) * 4;
                    if (accum) { o[0] += v[0]; o[1] += v[1]; o[2] += v[2]; o[3] += v[3]; }
                    else { o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3]; }
                }
            }
        }
    };

    if (lists) {
        // workgroup = 256 consecutive listed nodes of one z plane; a plane with more than
        // ntx * 256 listed nodes gives each of its workgroups further chunks, ntx apart
        const int lb = tl % ntx, z = tl / ntx;
        const int cnt = s.ccnt[pz_off + z];
        if (lb * 256 >= cnt) {
            if (s.pzmap[pz_off + z] >= 0 && threadIdx.x == 0) {
                double *o = s.pprt + (long long)g * s.nzt * 4;
                o[0] = 0.0; o[1] = 0.0; o[2] = 0.0; o[3] = 0.0;
            }
            return;
        }
        for (int lbx = lb; lbx * 256 < cnt; lbx += ntx) {
            const int kk = lbx * 256 + (int)threadIdx.x;
            const bool v = kk < cnt;
            const int c = v ? s.clist[cell_off + (long long)z * nxy + kk] - z * nxy : 0;
            // compact storage: the node's first link word (or the solid marker) at its slot
            const unsigned long long wcl = (CMP && v) ? s.lwc[cell_off + (long long)z * nxy + kk] : 0ull;
            const int jj = c / nx;
            const uint2 *lrt = nullptr;
            int jb = 0, nrows = 0;
            if constexpr (CMP) {
                // the chunk's nodes lie in rows jr[0] .. jr[1] (x-fastest list order): stage
                // the row-table words of their source rows once for the workgroup, unless
                // they do not fit (then each thread reads its own from the tables)
                const int last = min(cnt - lbx * 256, 256) - 1;
                if (threadIdx.x == 0) jr[0] = jj;
                if ((int)threadIdx.x == last) jr[1] = jj;
                __syncthreads();
                jb = jr[0] - 1;
                nrows = jr[1] - jr[0] + 3;
                const int tot = 3 * nrows * nw;
                if (tot <= kRtLds) {
                    const uint2 *rtab = s.rt + rt_off;
                    for (int w = threadIdx.x; w < tot; w += 256) {
                        const int pz = w / (nrows * nw), rem = w - pz * (nrows * nw);
                        const int u = rem / nw, wq = rem - u * nw;
                        const int zz = wrapc(z + pz - 1, nz), jg = wrapc(jb + u, ny);
                        rt_lds[w] = rtab[((long long)zz * ny + jg) * nw + wq];
                    }
                    lrt = rt_lds;
                }
                __syncthreads();
            }
            // the node's slot under compact storage
            run(c - jj * nx, jj, z, z + 1, z * nxy + kk, v, lbx != lb, lrt, jb, nrows, wcl);
            // (the next chunk stages its own rows once every thread is done with these)
            if constexpr (CMP) __syncthreads();
        }
    } else {
        const int bxl = uni(M->bx_log2);
        const int lx = threadIdx.x & ((1 << bxl) - 1), ly = threadIdx.x >> bxl;
        const int tx = tl % ntx, trem = tl / ntx, ty = trem % nty, tz = trem / nty;
        const int i = (tx << bxl) + lx;
        const int j = ty * uni(M->by) + ly;
        const int z0 = tz * s.nzt;
        run(i, j, z0, min(z0 + s.nzt, nz), 0, (i < nx) && (j < ny), false, nullptr, 0, 0, 0ull);
    }
}

// ---------------------------------------------------------------------------
// particle kernel: links, contacts, motion
// ---------------------------------------------------------------------------

// Node range [lo, lo + ext) along one axis covering [c - h, c + h]: clipped on a bounded
// axis, at most one full period on a periodic one.
__device__ __forceinline__ void axis_range(double c, double h, int n, int per, int &lo, int &ext)
{
    int l = (int)floor(c - h), u = (int)ceil(c + h);
    if (!per) { l = max(l, 0); u = min(u, n - 1); }
    else if (u - l + 1 > n) { l = 0; u = n - 1; }
    lo = l;
    ext = max(u - l + 1, 0);
}


// n / d for 0 <= n < 2^31 and a divisor d > 0 that every lane shares, through the FP64
// reciprocal (rounded within one unit of the quotient, then corrected)
__device__ __forceinline__ int div_uni(int n, int d, double inv)
{
    int q = (int)((double)n * inv);
    const int r = n - q * d;
    if (r < 0) q -= 1;
    else if (r >= d) q += 1;
    return q;
}

constexpr int kLinksBlock = 64;
constexpr int kLinkBatch = 2;
constexpr int kLinkScan = 4;  // shell cells per lane per scan round of a rebuilt chunk
// Direction masks over the links e (d = e*, c_d = -c_e), for sums over a node's links by
// counting: per axis and weight class (w = 1/18 on the axes, e < 6; 1/36 on the
// diagonals) the links whose c_d component is +1 or -1 ...
constexpr unsigned link_mask(int axis, int sign, bool diag)
{
    unsigned m = 0u;
    for (int e = 0; e < kQ - 1; ++e) {
        const int c = -(axis == 0 ? kCX[e] : axis == 1 ? kCY[e] : kCZ[e]);
        if (c == sign && (e >= 6) == diag) m |= 1u << e;
    }
    return m;
}
// ... and the diagonal links whose components along axes a and b have the product +1 or -1
constexpr unsigned pair_mask(int a, int b, int sign)
{
    unsigned m = 0u;
    for (int e = 6; e < kQ - 1; ++e) {
        const int ca = a == 0 ? kCX[e] : a == 1 ? kCY[e] : kCZ[e];
        const int cb = b == 0 ? kCX[e] : b == 1 ? kCY[e] : kCZ[e];
        if (ca * cb == sign) m |= 1u << e;
    }
    return m;
}

// Rebuild of one chunk of a particle's shell list (the wave of the calling lanes, for
// particle p): when the shell list was rebuilt, the node lists were rebuilt (storage slots
// move) or a node within one plane of the chunk's slab changed owner in the previous step,
// the chunk's entries that hold links of p are found again, compacted in list order, and
// its link-set sums recomputed; every other chunk keeps its entries.  It reads the link
// words of this step (after the refresh) and no link record: the record kernel runs it in
// waves of its own before its node waves, and the link pass reads the entries.
template <bool NR>
__device__ __forceinline__ void rebuild_chunk(const DevSet &s, int p, int chunk, long long t, int *lc, unsigned *lg)
{
    const int par = (int)(t & 1);
    const int lane = threadIdx.x & 63;
    // the chunk's state is loaded together with p's lattice, before the checks that need
    // the lattice (everything here is indexed by p < ptot)
    const int m = uni(s.pmem[p]);
    const double *Xo = s.X[par];
    const double X0 = Xo[3 * p], X1 = Xo[3 * p + 1], X2 = Xo[3 * p + 2];
    const int k0 = s.lchunk[p * (kChunks + 1) + chunk], k1 = s.lchunk[p * (kChunks + 1) + chunk + 1];
    // (a list rebuild under compact storage moves the nodes' storage slots)
    const bool fresh = (s.lreb[p] == t - 1) || (s.ldirty[p * kChunks + chunk] == t - 1) ||
                       (s.compact && *s.relist_at == t);
    if (!fresh) return;
    const MemberDev *M = s.mem + m;
    const int pl = p - uni(M->p_off);
    if (pl >= uni(M->np)) return;

    const int nx = uni(M->nx), ny = uni(M->ny);
    const int per0 = uni(M->per[0]), per1 = uni(M->per[1]), per2 = uni(M->per[2]);
    const double box0 = uni(M->box[0]), box1 = uni(M->box[1]), box2 = uni(M->box[2]);
    const long long cell_off = uni(M->cell_off);
    const double rho_f = uni(M->rho_f);
    const int nxy = nx * ny;
    const long long lbase = (long long)p * s.lcap;
    int *xc = s.xcell + lbase + k0;
    int *xs = s.xslot + lbase + k0;
    unsigned *xg = s.xgrp + lbase + k0;
    const double R0 = s.Xref[3 * p], R1 = s.Xref[3 * p + 1], R2 = s.Xref[3 * p + 2];
    const double inv_nxy = 1.0 / (double)nxy, inv_nx = 1.0 / (double)nx;

    // Link-set sums of a rebuilt chunk (the 6 x 6 matrix Z of the implicit update is
    // assembled from them): with S_n = sum over a node's links of 6 w_d rho_f c_d c_d^T and
    // xr its position relative to X_ref, S = sum S_n, Qx = sum [xr] S_n, Wx = sum [xr] S_n
    // [xr]^T ([v] the matrix of v x .).  On a lattice without narrow periodic axes they are
    // summed exactly, in integers, while the chunk's entries are found: S_n = z36 S'_n with
    // S'_n integer (6 w_d rho_f is 2 z36 on the axes and z36 on the diagonals), and xr = I -
    // fr with I the node's integer offset from floor(X_ref) (minimum image) and fr = X_ref -
    // floor(X_ref), so S = z36 sum S', Qx = z36 (sum [I] S' - [fr] sum S') and Wx = z36 (sum
    // [I] S' [I]^T - T - T^T + [fr] (sum S') [fr]^T), T = (sum [I] S') [fr]^T.  (|I| stays
    // below R + 3: the sums of S' and [I] S' fit 32 bits, those of [I] S' [I]^T take 64.)
    const int fl0 = (int)floor(R0), fl1 = (int)floor(R1), fl2 = (int)floor(R2);
    int zsi[15];
    long long zwl[6];
#pragma unroll
    for (int c = 0; c < 15; ++c) zsi[c] = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) zwl[c] = 0;
    auto add_link_set = [&](int cell, unsigned g) {
        const int kk = div_uni(cell, nxy, inv_nxy), rem = cell - kk * nxy;
        const int jj = div_uni(rem, nx, inv_nx), ii = rem - jj * nx;
        auto arm = [](int c, double R, int fl, int per, double box) {
            const double dx = (double)c - R;
            const int n = (int)box;
            return (c - fl) + ((per && dx > 0.5 * box) ? -n : ((per && dx < -0.5 * box) ? n : 0));
        };
        const int I0 = arm(ii, R0, fl0, per0, box0), I1 = arm(jj, R1, fl1, per1, box1), I2 = arm(kk, R2, fl2, per2, box2);
        auto diag = [&](int axis) {
            return 2 * (int)__popc(g & (link_mask(axis, 1, false) | link_mask(axis, -1, false))) +
                   (int)__popc(g & (link_mask(axis, 1, true) | link_mask(axis, -1, true)));
        };
        auto offd = [&](int a, int b2) {
            return (int)__popc(g & pair_mask(a, b2, 1)) - (int)__popc(g & pair_mask(a, b2, -1));
        };
        const int Sxx = diag(0), Syy = diag(1), Szz = diag(2);
        const int Sxy = offd(0, 1), Sxz = offd(0, 2), Syz = offd(1, 2);
        // [I] S' by columns (column n of S' is (S'_xn, S'_yn, S'_zn)), then row a of
        // [I] S' [I]^T as I x (row a of [I] S')
        // (24-bit multiplies: every factor is far below 2^23)
        auto cross = [](int a0, int a1, int a2, int b0, int b1, int b2, int &c0, int &c1, int &c2) {
            c0 = __mul24(a1, b2) - __mul24(a2, b1);
            c1 = __mul24(a2, b0) - __mul24(a0, b2);
            c2 = __mul24(a0, b1) - __mul24(a1, b0);
        };
        int q00, q10, q20, q01, q11, q21, q02, q12, q22;
        cross(I0, I1, I2, Sxx, Sxy, Sxz, q00, q10, q20);
        cross(I0, I1, I2, Sxy, Syy, Syz, q01, q11, q21);
        cross(I0, I1, I2, Sxz, Syz, Szz, q02, q12, q22);
        zsi[0] += Sxx; zsi[1] += Sxy; zsi[2] += Sxz; zsi[3] += Syy; zsi[4] += Syz; zsi[5] += Szz;
        zsi[6] += q00; zsi[7] += q01; zsi[8] += q02;
        zsi[9] += q10; zsi[10] += q11; zsi[11] += q12;
        zsi[12] += q20; zsi[13] += q21; zsi[14] += q22;
        int w00, w01, w02, w10, w11, w12, w20, w21, w22;
        cross(I0, I1, I2, q00, q01, q02, w00, w01, w02);
        cross(I0, I1, I2, q10, q11, q12, w10, w11, w12);
        cross(I0, I1, I2, q20, q21, q22, w20, w21, w22);
        (void)w10; (void)w20; (void)w21;
        zwl[0] += w00; zwl[1] += w01; zwl[2] += w02; zwl[3] += w11; zwl[4] += w12; zwl[5] += w22;
    };

    // (1) the chunk's shell-list entries that hold links of p, compacted in list order;
    // kept from the previous step unless the list was rebuilt or a node within one plane
    // of the chunk's slab changed owner in the previous step (the refresh of this step
    // has brought the link words up to date)
    int cntx = 0;
    {
        // kLinkScan cells per lane and round: their list masks and cells, then their link
        // words, then the second words and storage slots are loaded in three rounds
        // instead of three per cell; the cells are then taken in list order
        for (int base = k0; base < k1; base += kLinksBlock * kLinkScan) {
            unsigned mk[kLinkScan];
            int cl[kLinkScan];
#pragma unroll
            for (int b = 0; b < kLinkScan; ++b) {
                const int k = base + b * kLinksBlock + lane;
                // (every lane loads: past the chunk's end it reads the chunk's first entry)
                const int kc = k < k1 ? k : k0;
                const unsigned mkr = s.lmask[lbase + kc];
                const int clr = s.lcell[lbase + kc];
                mk[b] = k < k1 ? mkr : 0u;
                cl[b] = k < k1 ? clr : 0;
            }
            unsigned long long w0b[kLinkScan];
#pragma unroll
            for (int b = 0; b < kLinkScan; ++b) {
                const unsigned long long wr = s.lw[cell_off + cl[b]];
                w0b[b] = mk[b] != 0u ? wr : 0ull;
            }
            unsigned long long w1b[kLinkScan];
            int nsb[kLinkScan];
#pragma unroll
            for (int b = 0; b < kLinkScan; ++b) {
                if (((unsigned)w0b[b] & 0x3ffffu) == 0u) w0b[b] = 0ull;
                w1b[b] = (w0b[b] >> 62) ? s.lw[s.ncell_total + cell_off + cl[b]] : 0ull;
                {
                    const int cell = cl[b], kk = div_uni(cell, nxy, inv_nxy), rem = cell - kk * nxy;
                    const int jj = div_uni(rem, nx, inv_nx);
                    const int ns = node_slot(s, M, cell, rem - jj * nx, jj, kk);
                    nsb[b] = w0b[b] != 0ull ? ns : 0;
                }
            }
#pragma unroll
            for (int b = 0; b < kLinkScan; ++b) {
                const int cell = cl[b];
                const unsigned long long w0 = w0b[b], w1 = w1b[b];
                const int ng = (w0 >> 62) ? 4 : 2;
                // one entry per slot of p at the node: one pass, or more in a set with a
                // narrow lattice, where a node can hold links into two images of p (one slot
                // each)
                int g0 = 0;
                for (int pass = 0; pass < (NR ? 4 : 1); ++pass) {
                    unsigned grp = 0u;
                    int slot = 0;
                    for (int g = g0; g < ng; ++g) {
                        int q;
                        const unsigned gd = slot_dirs(w0, w1, g, q);
                        if (gd != 0u && q == pl) { grp = gd; slot = g; break; }
                    }
                    const bool has = grp != 0u;
                    const unsigned long long bal = __ballot(has);
                    if (bal == 0ull) break;
                    if (has) {
                        const int at = cntx + __popcll(bal & ((1ull << lane) - 1ull));
                        if (at < k1 - k0) {
                            xc[at] = (int)((unsigned)cell | ((unsigned)slot << 30));
                            xs[at] = nsb[b];
                            xg[at] = grp;
                            // (the first kLinkLds entries also in this wave's LDS, where the
                            // link-set sums read them)
                            if (at < kLinkLds) {
                                lc[at] = (int)((unsigned)cell | ((unsigned)slot << 30));
                                lg[at] = grp;
                            }
                        } else {
                            atomicOr(s.flags, 0x40u);
                        }
                        g0 = slot + 1;
                    } else {
                        g0 = ng;
                    }
                    cntx = min(cntx + __popcll(bal), k1 - k0);
                }
            }
        }
        if (lane == 0) s.xcnt[p * kChunks + chunk] = cntx;
        // (the link-set sums read the entries back, from LDS, or from memory for a chunk
        // with more than kLinkLds entries: the wave's writes are made visible to the wave
        // itself; the other waves of its workgroup rebuild other chunks)
        if (cntx <= kLinkLds) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
    }
    const bool from_lds = cntx <= kLinkLds;


    // Positions of the entries' nodes relative to the shell list's reference point X_ref,
    // xr = x - X_ref (minimum image; X_ref moves only when the shell list is rebuilt, which
    // rebuilds the entries).  With delta = X - X_ref, r = xr - delta, so the torque is
    // sum xr x G - delta x F0, and Z follows from sums over the link set alone:
    // S = sum S_n, Qx = sum [xr] S_n, Wx = sum [xr] S_n [xr]^T (the motion kernel applies delta).
    const double z18 = rho_f / 3.0, z36 = rho_f / 6.0;                  // 6 rho_f w_d
    // (in a set with a narrow lattice the entry's image of p is the one that holds its link
    // group: its arm from the current centre X, as group_arm, plus the small displacement
    // X - X_ref)
    const double dX0 = mimg(X0 - R0, per0, box0), dX1 = mimg(X1 - R1, per1, box1), dX2 = mimg(X2 - R2, per2, box2);
    auto rel_pos = [&](int cell, unsigned g, double &x0, double &x1, double &x2) {
        const int kk = div_uni(cell, nxy, inv_nxy), rem = cell - kk * nxy;
        const int jj = div_uni(rem, nx, inv_nx), ii = rem - jj * nx;
        if constexpr (NR) {
            group_arm<true>(M, g, ii, jj, kk, X0, X1, X2, x0, x1, x2);
            x0 += dX0; x1 += dX1; x2 += dX2;
        } else {
            x0 = mimg((double)ii - R0, per0, box0);
            x1 = mimg((double)jj - R1, per1, box1);
            x2 = mimg((double)kk - R2, per2, box2);
        }
    };

    // (2) link-set sums of a rebuilt chunk: S, Qx, Wx (21 values, cached per chunk); exact
    // integer sums from the scan, or, in a set with a narrow lattice, FP64 sums over the
    // entries in list order
    if (!NR) {
        if (from_lds)
            for (int k = lane; k < cntx; k += kLinksBlock) add_link_set((int)((unsigned)lc[k] & 0x3fffffffu), lg[k]);
        else
            for (int k = lane; k < cntx; k += kLinksBlock) add_link_set((int)((unsigned)xc[k] & 0x3fffffffu), xg[k]);
        int si[15];
#pragma unroll
        for (int c = 0; c < 15; ++c) si[c] = wave_sum_i(zsi[c]);
        double wl[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) wl[c] = wave_sum((double)zwl[c]); // exact: integers below 2^53
        if (lane == 0) {
            const double f0 = R0 - (double)fl0, f1 = R1 - (double)fl1, f2 = R2 - (double)fl2;
            double Ss[3][3], Qs[3][3], Ws[3][3];
            {
                int z = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = a; c < 3; ++c) { Ss[a][c] = (double)si[z]; Ss[c][a] = (double)si[z]; ++z; }
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) Qs[a][c] = (double)si[z++];
                z = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = a; c < 3; ++c) { Ws[a][c] = wl[z]; Ws[c][a] = wl[z]; ++z; }
            }
            // fr x (column n of M) for M = sum S'; fr x (row a of M) for M = sum [I] S' and
            // for M = [fr] sum S'
            double FS[3][3], T[3][3], FSF[3][3];
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                FS[0][n] = f1 * Ss[2][n] - f2 * Ss[1][n];
                FS[1][n] = f2 * Ss[0][n] - f0 * Ss[2][n];
                FS[2][n] = f0 * Ss[1][n] - f1 * Ss[0][n];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                T[a][0] = f1 * Qs[a][2] - f2 * Qs[a][1];
                T[a][1] = f2 * Qs[a][0] - f0 * Qs[a][2];
                T[a][2] = f0 * Qs[a][1] - f1 * Qs[a][0];
                FSF[a][0] = f1 * FS[a][2] - f2 * FS[a][1];
                FSF[a][1] = f2 * FS[a][0] - f0 * FS[a][2];
                FSF[a][2] = f0 * FS[a][1] - f1 * FS[a][0];
            }
            double *zc = s.zcache + ((long long)p * kChunks + chunk) * kZComp;
            int z = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = a; c < 3; ++c) zc[z++] = z36 * Ss[a][c];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) zc[z++] = z36 * (Qs[a][c] - FS[a][c]);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = a; c < 3; ++c) zc[z++] = z36 * (((Ws[a][c] - T[a][c]) - T[c][a]) + FSF[a][c]);
        }
    }
    if (NR) {
        double zs[21];
#pragma unroll
        for (int c = 0; c < 21; ++c) zs[c] = 0.0;
        for (int k = lane; k < cntx; k += kLinksBlock) {
            const unsigned g = from_lds ? lg[k] : xg[k];
            double x0, x1, x2;
            rel_pos((int)((unsigned)(from_lds ? lc[k] : xc[k]) & 0x3fffffffu), g, x0, x1, x2);
            // S_n = sum 6 w_d rho_f c_d c_d^T over the node's links, from counts
            auto diag = [&](int axis) {
                return z18 * (double)__popc(g & (link_mask(axis, 1, false) | link_mask(axis, -1, false))) +
                       z36 * (double)__popc(g & (link_mask(axis, 1, true) | link_mask(axis, -1, true)));
            };
            auto offd = [&](int a, int b2) {
                // (the counts are unsigned: take the difference as a signed integer)
                const int n = (int)__popc(g & pair_mask(a, b2, 1)) - (int)__popc(g & pair_mask(a, b2, -1));
                return z36 * (double)n;
            };
            const double Sxy = offd(0, 1), Sxz = offd(0, 2), Syz = offd(1, 2);
            const double Sm[3][3] = {{diag(0), Sxy, Sxz}, {Sxy, diag(1), Syz}, {Sxz, Syz, diag(2)}};
            // Q = [xr] S_n (row a: xr x (column of S_n)), W = Q [xr]^T
            double Qm[3][3], Wm[3][3];
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                Qm[0][n] = x1 * Sm[2][n] - x2 * Sm[1][n];
                Qm[1][n] = x2 * Sm[0][n] - x0 * Sm[2][n];
                Qm[2][n] = x0 * Sm[1][n] - x1 * Sm[0][n];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Wm[a][0] = x1 * Qm[a][2] - x2 * Qm[a][1];
                Wm[a][1] = x2 * Qm[a][0] - x0 * Qm[a][2];
                Wm[a][2] = x0 * Qm[a][1] - x1 * Qm[a][0];
            }
            int z = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b2 = a; b2 < 3; ++b2) zs[z++] += Sm[a][b2];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b2 = 0; b2 < 3; ++b2) zs[z++] += Qm[a][b2];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b2 = a; b2 < 3; ++b2) zs[z++] += Wm[a][b2];
        }
#pragma unroll
        for (int c = 0; c < 21; ++c) zs[c] = wave_sum(zs[c]);
        if (lane == 0) {
            double *zc = s.zcache + ((long long)p * kChunks + chunk) * kZComp;
#pragma unroll
            for (int c = 0; c < 21; ++c) zc[c] = zs[c];
        }
    }

}

// Link pass, one wave per (particle p, chunk of p's shell list).  A link of p is a fluid
// node x and a direction e whose source x - c_e lies in p; with d = e* pointing into p,
// Eq. (fFS) with Eq. (mem) substituted gives
//   F = c_d f~_d(x,t) - c_e f_e(x,t+1) = 2 c_d f~_d(x,t) - (2 w_d / c_s^2) rho_f c_d (c_d . V_b),
// V_b = V_p + Omega_p x (x_b - X_p), x_b = x + c_d/2.  Since (x_b - X_p) x c_d = (x - X_p) x c_d
// = r x c_d, the force and its torque about X_p over the step are (F, T) = F0 - Z (V, Omega)
// with F0 = (G, r x G), G = sum 2 c_d f~_d(x,t), and Z = sum (2 w_d / c_s^2) rho_f a_d a_d^T,
// a_d = (c_d, r x c_d).  Per node, with S = sum over its links to p of 6 w_d rho_f c_d c_d^T
// and [r] the matrix of r x .: Z_VV = S, Z_OmegaV = [r] S, Z_OmegaOmega = [r] S [r]^T.  G is
// summed from the deviations f~_d - w_d rho_f (the rest part 2 rho_f sum w_d c_d and S come
// from counts of links per direction class), the sums over the chunk in FP64 in a fixed
// order; the motion kernel adds the chunks in chunk order and solves for (V, Omega).
// The deviation sums of a node's links come from the record k_records wrote for the node's
// slot in this step.
template <int P, bool NR>
__global__ __launch_bounds__(kLinksBlock) void k_links(DevSet s, int mode, int only)
{
    const long long t = *s.tstep;
    const int par = (int)(t & 1);
    const int lane = threadIdx.x;
    const int p = blockIdx.x / kChunks, chunk = blockIdx.x - p * kChunks;
    if (p >= s.ptot || mode != 0) return;
    // the chunk's state is loaded together with p's lattice, before the checks that need
    // the lattice (everything here is indexed by p < ptot)
    const int m = uni(s.pmem[p]);
    const double *Xo = s.X[par];
    const double X0 = Xo[3 * p], X1 = Xo[3 * p + 1], X2 = Xo[3 * p + 2];
    const int k0 = s.lchunk[p * (kChunks + 1) + chunk], k1 = s.lchunk[p * (kChunks + 1) + chunk + 1];
    // the chunk's entries (rebuilt by the record kernel of this step where they changed)
    const int cntx = s.xcnt[p * kChunks + chunk];
    const MemberDev *M = s.mem + m;
    const int pl = p - uni(M->p_off);
    if (pl >= uni(M->np)) return;
    if (only >= 0 && m != only) return;

    const int nx = uni(M->nx), ny = uni(M->ny);
    const int per0 = uni(M->per[0]), per1 = uni(M->per[1]), per2 = uni(M->per[2]);
    const double box0 = uni(M->box[0]), box1 = uni(M->box[1]), box2 = uni(M->box[2]);
    const long long cell_off = uni(M->cell_off);
    const double rho_f = uni(M->rho_f);
    const bool rest_free = uni(M->rest_free) != 0;
    const int nxy = nx * ny;
    const long long lbase = (long long)p * s.lcap;
    const int *xc = s.xcell + lbase + k0;
    const int *xs = s.xslot + lbase + k0;
    const unsigned *xg = s.xgrp + lbase + k0;
    const double R0 = s.Xref[3 * p], R1 = s.Xref[3 * p + 1], R2 = s.Xref[3 * p + 2];
    const double inv_nxy = 1.0 / (double)nxy, inv_nx = 1.0 / (double)nx;


    // Positions of the entries' nodes relative to the shell list's reference point X_ref,
    // xr = x - X_ref (minimum image; X_ref moves only when the shell list is rebuilt, which
    // rebuilds the entries).  With delta = X - X_ref, r = xr - delta, so the torque is
    // sum xr x G - delta x F0, and Z follows from sums over the link set alone:
    // S = sum S_n, Qx = sum [xr] S_n, Wx = sum [xr] S_n [xr]^T (the motion kernel applies delta).
    const double a18 = 2.0 * rho_f / 18.0, a36 = 2.0 * rho_f / 36.0;   // 2 rho_f w_d
    // (in a set with a narrow lattice the entry's image of p is the one that holds its link
    // group: its arm from the current centre X, as group_arm, plus the small displacement
    // X - X_ref)
    const double dX0 = mimg(X0 - R0, per0, box0), dX1 = mimg(X1 - R1, per1, box1), dX2 = mimg(X2 - R2, per2, box2);
    auto rel_pos = [&](int cell, unsigned g, double &x0, double &x1, double &x2) {
        const int kk = div_uni(cell, nxy, inv_nxy), rem = cell - kk * nxy;
        const int jj = div_uni(rem, nx, inv_nx), ii = rem - jj * nx;
        if constexpr (NR) {
            group_arm<true>(M, g, ii, jj, kk, X0, X1, X2, x0, x1, x2);
            x0 += dX0; x1 += dX1; x2 += dX2;
        } else {
            x0 = mimg((double)ii - R0, per0, box0);
            x1 = mimg((double)jj - R1, per1, box1);
            x2 = mimg((double)kk - R2, per2, box2);
        }
    };

    // (3) F0 = sum 2 c_d f~_d and sum xr x (the node's part of F0) over the entries
    double acc[kLinkComp];
#pragma unroll
    for (int c = 0; c < kLinkComp; ++c) acc[c] = 0.0;
    for (int base = 0; base < cntx; base += kLinksBlock * kLinkBatch) {
        int cellb[kLinkBatch];
        unsigned gb[kLinkBatch];
        // (records are kept in the collision precision until they are summed)
        typename Prec<P>::C Db[kLinkBatch][3];
#pragma unroll
        for (int b = 0; b < kLinkBatch; ++b) {
            const int k = base + b * kLinksBlock + lane;
            const bool v = k < cntx;
            const int kv = v ? k : 0;
            const unsigned ent = v ? (unsigned)xc[kv] : 0u;
            cellb[b] = (int)(ent & 0x3fffffffu);
            // (a node with links is fluid, hence listed; entries past the count read the
            // first record and carry no directions)
            const int xsr = xs[kv];
            const unsigned xgr = xg[kv];
            const int at = v ? max(xsr, 0) : 0;
            gb[b] = v ? xgr : 0u;
            if constexpr (sizeof(typename Prec<P>::C) == 4) {
                const float4 v4 = reinterpret_cast<const float4 *>(s.frec)[(int)(ent >> 30) * s.ncell_total + cell_off + at];
                Db[b][0] = v4.x; Db[b][1] = v4.y; Db[b][2] = v4.z;
            } else {
                double G0, G1, G2;
                (void)get_record<P>(s, (int)(ent >> 30), cell_off + at, G0, G1, G2);
                Db[b][0] = G0; Db[b][1] = G1; Db[b][2] = G2;
            }
        }
#pragma unroll
        for (int b = 0; b < kLinkBatch; ++b) {
            const unsigned g = gb[b];
            if (g == 0u) continue;
            // G = sum 2 c_d (f~_d - w_d rho_f) + 2 rho_f sum w_d c_d
            auto rest = [&](int axis) {
                const int na = (int)__popc(g & link_mask(axis, 1, false)) - (int)__popc(g & link_mask(axis, -1, false));
                const int nd = (int)__popc(g & link_mask(axis, 1, true)) - (int)__popc(g & link_mask(axis, -1, true));
                return a18 * (double)na + a36 * (double)nd;
            };
            // (rest_free: without the rest state's part)
            const double G0 = 2.0 * (double)Db[b][0] + (rest_free ? 0.0 : rest(0));
            const double G1 = 2.0 * (double)Db[b][1] + (rest_free ? 0.0 : rest(1));
            const double G2 = 2.0 * (double)Db[b][2] + (rest_free ? 0.0 : rest(2));
            double x0, x1, x2;
            rel_pos(cellb[b], g, x0, x1, x2);
            acc[0] += G0; acc[1] += G1; acc[2] += G2;
            acc[3] += x1 * G2 - x2 * G1;
            acc[4] += x2 * G0 - x0 * G2;
            acc[5] += x0 * G1 - x1 * G0;
        }
    }
#pragma unroll
    for (int c = 0; c < kLinkComp; ++c) acc[c] = wave_sum(acc[c]);
    if (lane == 0) {
        double *pp = s.ppart + ((long long)p * kChunks + chunk) * kLinkComp;
#pragma unroll
        for (int c = 0; c < kLinkComp; ++c) pp[c] = acc[c];
    }
}

// Solves A x = b for a symmetric positive definite 6 x 6 A (upper triangle given) by the
// factorisation A = L D L^T (L unit lower triangular, D diagonal), with one division per
// pivot; b is overwritten by x.
__device__ __forceinline__ void ldl_solve6(double (&A)[6][6], double (&b)[6])
{
    double L[6][6], E[6][6], iD[6]; // E[i][j] = L[i][j] D[j]
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * E[j][k];
        iD[j] = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double v = A[j][i];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= L[i][k] * E[j][k];
            E[i][j] = v;
            L[i][j] = v * iD[j];
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double v = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[i][k] * b[k];
        b[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) b[i] *= iD[i];
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double v = b[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) v -= L[k][i] * b[k];
        b[i] = v;
    }
}

// One wave per particle, kMotionWaves particles per workgroup.
// mode 0: Eqs. (translate), (rotate) over the step with symplectic Euler, dt = 1: Hertz /
//         Mindlin contacts (Eqs. fdLawn, fdLaws) with the particles of the near list at
//         X(t), V(t), the external force, the conversion impulses of the previous
//         re-projection, and the momentum exchanged with the fluid in this step, F0 - Z
//         (V', Omega') from the link pass (chunk partials summed in chunk order), solved
//         for the velocities of the step, (M + Z)(V', Omega') = M (V, Omega) + F0 + the
//         rest; X(t+1) = X(t) + V'.  F_h, T_h of Eqs. (coupleF), (coupleT) are reported.
//         Fixed particles stay.  The fluid kernel's wall state (X(t), V', Omega') is
//         written in FP32.
// mode 1: near-neighbour list (every particle within R_p + R_q + kNearMargin) and the FP32
//         state copy (set-up); later lists are built by the re-projection kernel.
constexpr int kMotionWaves = 4;
__global__ __launch_bounds__(64 * kMotionWaves) void k_motion(DevSet s, int mode, int only)
{
    const long long t = *s.tstep;
    const int par = (int)(t & 1);
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * kMotionWaves + (int)(threadIdx.x >> 6);
    if (p >= s.ptot) return; // the whole wave: waves never synchronise here
    // p's state, its link-pass sums and its near list are loaded together, before the
    // checks that need its lattice (everything here is indexed by p < ptot)
    const int m = s.pmem[p];
    const double *Xo = s.X[par], *Vo = s.V[par], *Wo = s.W[par];
    const double X0 = Xo[3 * p], X1 = Xo[3 * p + 1], X2 = Xo[3 * p + 2];
    const double R = s.R[p];
    // the link pass's sums (lane c < kLinkComp adds component c of the partials over the
    // chunks, lane kLinkComp + c component c of the cached link-set sums, in chunk order)
    // and the rest of p's state for the update, loaded up front
    static_assert(kLinkComp + kZComp <= 64, "one lane per link-pass component");
    // (with the hydrodynamics switched off there are neither link forces nor conversion
    // momenta)
    const bool hyd = !s.fluid_off;
    double ppv = 0.0;
    if (mode == 0 && hyd && lane < kLinkComp + kZComp) {
        const bool part = lane < kLinkComp;
        const int stride = part ? kLinkComp : kZComp;
        const double *pp = part ? s.ppart + (long long)p * kChunks * kLinkComp + lane
                                : s.zcache + (long long)p * kChunks * kZComp + (lane - kLinkComp);
        double ch[kChunks];
#pragma unroll
        for (int q = 0; q < kChunks; ++q) ch[q] = pp[q * stride];
#pragma unroll
        for (int q = 0; q < kChunks; ++q) ppv += ch[q];
    }
    const double Xr0 = s.Xref[3 * p], Xr1 = s.Xref[3 * p + 1], Xr2 = s.Xref[3 * p + 2];
    double Phv[3], Lhv[3], Fgv[3], Vpv[3], Wpv[3];
    for (int a = 0; a < 3; ++a) {
        Phv[a] = hyd ? s.Ph[3 * p + a] : 0.0;
        Lhv[a] = hyd ? s.Lh[3 * p + a] : 0.0;
        Fgv[a] = s.Fg[3 * p + a];
        Vpv[a] = Vo[3 * p + a];
        Wpv[a] = Wo[3 * p + a];
    }
    const double mass = s.m[p], inert = s.I[p];
    const int fixed_p = s.fixed[p];
    const int nn_ld = s.nnear[p];
    const int *nl = s.nearl + (long long)p * kNearCap;
    const int nl_ld = nl[lane & (kNearCap - 1)];
    const int hno = s.hn[par][p];
    const MemberDev *M = s.mem + m;
    if (p - M->p_off >= M->np) return;
    if (only >= 0 && m != only) return;
    const int per0 = M->per[0], per1 = M->per[1], per2 = M->per[2];
    const double box0 = M->box[0], box1 = M->box[1], box2 = M->box[2];

    // contacts over the near list (mode 0) or the near-list build (mode 1)
    const int q0 = M->p_off, nq = M->np;
    const double E = M->E, nu = M->nu, mu = M->mu;
    const int *hjo = s.hj[par] + (long long)p * kHistCap;
    const double *hfo = s.hf[par] + (long long)p * kHistCap * 3;
    int *hjn = s.hj[par ^ 1] + (long long)p * kHistCap;
    double *hfn = s.hf[par ^ 1] + (long long)p * kHistCap * 3;
    double con[6] = {0, 0, 0, 0, 0, 0};
    int near_total = 0, hist_total = 0;
    const bool build = mode != 0;
    const int ncand = build ? nq : min(nn_ld, kNearCap);
    const unsigned long long below = (1ull << lane) - 1ull;
    static_assert(kNearCap <= 64, "a near list fits one wave");
    for (int base = 0; base < ncand; base += 64) {
        const int jj = base + lane;
        // (a near list has at most kNearCap <= 64 entries: lane jj < ncand took entry jj)
        const int q = (jj < ncand) ? (build ? q0 + jj : nl_ld) : -1;
        bool isnear = false, keep = false;
        double ftn[3] = {0, 0, 0};
        if (jj < ncand && q != p) {
            const double Y0 = Xo[3 * q], Y1 = Xo[3 * q + 1], Y2 = Xo[3 * q + 2], Rq = s.R[q];
            const double d0 = mimg(Y0 - X0, per0, box0);
            const double d1 = mimg(Y1 - X1, per1, box1);
            const double d2 = mimg(Y2 - X2, per2, box2);
            const double dist = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
            isnear = dist <= R + Rq + kNearMargin;
            const double un = R + Rq - dist;
            if (mode == 0 && un > 0.0) {
                // Eq. (fdLawn): Hertz normal force, pushing p away from q
                const double n0 = d0 / dist, n1 = d1 / dist, n2 = d2 / dist;
                const double rstar = 1.0 / (1.0 / R + 1.0 / Rq);
                const double fn = 2.0 * E * un * sqrt(rstar * un) / (3.0 * (1.0 - nu * nu));
                con[0] += -fn * n0; con[1] += -fn * n1; con[2] += -fn * n2;
                if (mu > 0.0) {
                    // Eq. (fdLaws): incremental Mindlin spring, Coulomb cap
                    double fo[3] = {0, 0, 0};
                    for (int h = 0; h < hno; ++h)
                        if (hjo[h] == q) { fo[0] = hfo[3 * h]; fo[1] = hfo[3 * h + 1]; fo[2] = hfo[3 * h + 2]; }
                    const double a0 = (R - 0.5 * un) * n0, a1 = (R - 0.5 * un) * n1, a2 = (R - 0.5 * un) * n2;
                    const double b0 = -(Rq - 0.5 * un) * n0, b1 = -(Rq - 0.5 * un) * n1, b2 = -(Rq - 0.5 * un) * n2;
                    const double *Vq = Vo + 3 * q, *Wq = Wo + 3 * q, *Vp = Vo + 3 * p, *Wp = Wo + 3 * p;
                    const double wa0 = Wp[1] * a2 - Wp[2] * a1, wa1 = Wp[2] * a0 - Wp[0] * a2, wa2 = Wp[0] * a1 - Wp[1] * a0;
                    const double wb0 = Wq[1] * b2 - Wq[2] * b1, wb1 = Wq[2] * b0 - Wq[0] * b2, wb2 = Wq[0] * b1 - Wq[1] * b0;
                    const double v0 = (Vp[0] + wa0) - (Vq[0] + wb0);
                    const double v1 = (Vp[1] + wa1) - (Vq[1] + wb1);
                    const double v2 = (Vp[2] + wa2) - (Vq[2] + wb2);
                    const double vn = v0 * n0 + v1 * n1 + v2 * n2;
                    const double fon = fo[0] * n0 + fo[1] * n1 + fo[2] * n2;
                    const double kt = 2.0 * E * sqrt(rstar * un) / ((1.0 + nu) * (2.0 - nu));
                    ftn[0] = (fo[0] - fon * n0) - kt * (v0 - vn * n0);
                    ftn[1] = (fo[1] - fon * n1) - kt * (v1 - vn * n1);
                    ftn[2] = (fo[2] - fon * n2) - kt * (v2 - vn * n2);
                    const double fm = sqrt(ftn[0] * ftn[0] + ftn[1] * ftn[1] + ftn[2] * ftn[2]);
                    if (fm > mu * fn) { const double sc = mu * fn / fm; ftn[0] *= sc; ftn[1] *= sc; ftn[2] *= sc; }
                    con[0] += ftn[0]; con[1] += ftn[1]; con[2] += ftn[2];
                    con[3] += a1 * ftn[2] - a2 * ftn[1];
                    con[4] += a2 * ftn[0] - a0 * ftn[2];
                    con[5] += a0 * ftn[1] - a1 * ftn[0];
                    keep = true;
                }
            }
        }
        if (build) {
            const unsigned long long bal = __ballot(isnear);
            if (isnear) {
                const int slot = near_total + __popcll(bal & below);
                if (slot < kNearCap) s.nearl[(long long)p * kNearCap + slot] = q;
                else atomicOr(s.flags, 0x2u);
            }
            near_total += __popcll(bal);
        }
        if (mode == 0 && mu > 0.0) {
            const unsigned long long bal = __ballot(keep);
            if (keep) {
                const int slot = hist_total + __popcll(bal & below);
                if (slot < kHistCap) {
                    hjn[slot] = q;
                    hfn[3 * slot] = ftn[0]; hfn[3 * slot + 1] = ftn[1]; hfn[3 * slot + 2] = ftn[2];
                } else {
                    atomicOr(s.flags, 0x8u);
                }
            }
            hist_total += __popcll(bal);
        }
    }
    if (lane == 0) {
        if (build) {
            s.nnear[p] = min(near_total, kNearCap);
            s.near_at[p] = t;
        }
        if (mode == 0) s.hn[par ^ 1][p] = min(hist_total, kHistCap);
    }
    if (mode != 0) {
        if (lane == 0) pack_state(s.pf[par] + 12 * p, Xo + 3 * p, Vo + 3 * p, Wo + 3 * p);
        return;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) con[c] = wave_sum(con[c]);

    // the link pass's sums (every lane takes the same values): F0, sum xr x G, then the
    // link-set sums S, Qx, Wx
    double lp[kLinkComp + kZComp];
#pragma unroll
    for (int c = 0; c < kLinkComp + kZComp; ++c) lp[c] = readlane_d(ppv, c);
    if (lane == 0) {
        double *Xn = s.X[par ^ 1], *Vn = s.V[par ^ 1], *Wn = s.W[par ^ 1];
        const double Xc[3] = {X0, X1, X2};
        const int per[3] = {per0, per1, per2};
        const double box[3] = {box0, box1, box2};
        // delta = X - X_ref: the torque arm of a link node is xr - delta
        const double dl[3] = {mimg(X0 - Xr0, per0, box0), mimg(X1 - Xr1, per1, box1), mimg(X2 - Xr2, per2, box2)};
        // T0 = sum xr x G - delta x F0
        lp[3] -= dl[1] * lp[2] - dl[2] * lp[1];
        lp[4] -= dl[2] * lp[0] - dl[0] * lp[2];
        lp[5] -= dl[0] * lp[1] - dl[1] * lp[0];
        // Z: Z_VV = S, Z_OmegaV = Qx - [delta] S, Z_OmegaOmega = Wx - Qx [delta]^T - [delta] Qx^T
        // + [delta] S [delta]^T, with [delta] v = delta x v
        double Sm[3][3], Qm[3][3], Wm[3][3];
        {
            const double *zz = lp + kLinkComp;
            int z = 0;
            for (int a = 0; a < 3; ++a)
                for (int c = a; c < 3; ++c) { Sm[a][c] = zz[z]; Sm[c][a] = zz[z]; ++z; }
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) Qm[a][c] = zz[z++];
            for (int a = 0; a < 3; ++a)
                for (int c = a; c < 3; ++c) { Wm[a][c] = zz[z]; Wm[c][a] = zz[z]; ++z; }
        }
        const double Dm[3][3] = {{0.0, -dl[2], dl[1]}, {dl[2], 0.0, -dl[0]}, {-dl[1], dl[0], 0.0}};
        double DS[3][3], ZOV[3][3], ZOO[3][3];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                double v = 0.0;
                for (int k = 0; k < 3; ++k) v += Dm[a][k] * Sm[k][c];
                DS[a][c] = v;
                ZOV[a][c] = Qm[a][c] - v;
            }
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                double qd = 0.0, dq = 0.0, dsd = 0.0;
                for (int k = 0; k < 3; ++k) {
                    qd += Qm[a][k] * Dm[c][k];
                    dq += Dm[a][k] * Qm[c][k];
                    dsd += DS[a][k] * Dm[c][k];
                }
                ZOO[a][c] = ((Wm[a][c] - qd) - dq) + dsd;
            }
        // (M + Z)(V', Omega') = M (V, Omega) + F0 + contacts + F_g + pending impulses; Z's
        // upper triangle: rows 0-2 (V) S and Z_VOmega = Z_OmegaV^T, rows 3-5 Z_OmegaOmega
        double A[6][6], b[6];
        double zup[21];
        {
            int z = 0;
            for (int a = 0; a < 3; ++a) {
                for (int c = a; c < 3; ++c) A[a][c] = Sm[a][c];
                for (int c = 0; c < 3; ++c) A[a][3 + c] = ZOV[c][a];
            }
            for (int a = 0; a < 3; ++a)
                for (int c = a; c < 3; ++c) A[3 + a][3 + c] = ZOO[a][c];
            for (int a = 0; a < 6; ++a)
                for (int c = a; c < 6; ++c) zup[z++] = A[a][c];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            A[a][a] += mass;
            A[3 + a][3 + a] += inert;
            b[a] = mass * Vpv[a] + (((lp[a] + Phv[a]) + Fgv[a]) + con[a]);
            b[3 + a] = inert * Wpv[a] + ((lp[3 + a] + Lhv[a]) + con[3 + a]);
        }
        double x[6] = {b[0], b[1], b[2], b[3], b[4], b[5]};
        ldl_solve6(A, x);
        double v[3] = {x[0], x[1], x[2]}, w[3] = {x[3], x[4], x[5]};
        if (fixed_p) {
            for (int a = 0; a < 3; ++a) { v[a] = 0.0; w[a] = 0.0; }
        } else {
            // a step beyond 0.25 lu (or a non-finite state) is an error (status 0x10); the
            // particle is then held to a step of 0.25 lu and inside the lattice, so that
            // every index derived from its position stays in range
            const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            const bool fin = isfinite(v2) && isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2]);
            if (!fin || !(v2 <= 0.0625)) {
                atomicOr(s.flags, 0x10u);
                if (!fin) {
                    for (int a = 0; a < 3; ++a) { v[a] = 0.0; w[a] = 0.0; }
                } else {
                    const double sc = 0.25 / sqrt(v2);
                    for (int a = 0; a < 3; ++a) v[a] *= sc;
                }
            }
        }
        // F_h, T_h: the momentum exchanged with the fluid over the step, F0 - Z (V', Omega'),
        // plus the pending impulses used here (Eqs. coupleF, coupleT)
        const double xv[6] = {v[0], v[1], v[2], w[0], w[1], w[2]};
        double zx[6] = {0, 0, 0, 0, 0, 0};
        {
            int z = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int c = a; c < 6; ++c) {
                    const double zz = zup[z++];
                    zx[a] += zz * xv[c];
                    if (c != a) zx[c] += zz * xv[a];
                }
        }
        for (int a = 0; a < 3; ++a) {
            s.Fh[3 * p + a] = (lp[a] - zx[a]) + Phv[a];
            s.Th[3 * p + a] = (lp[3 + a] - zx[3 + a]) + Lhv[a];
        }
        if (s.pv_ring > 0) {
            double *pv = s.pvring + ((t % s.pv_ring) * (long long)s.ptot + p) * 3;
            pv[0] = v[0]; pv[1] = v[1]; pv[2] = v[2];
        }
        for (int a = 0; a < 3; ++a) {
            Vn[3 * p + a] = v[a];
            Wn[3 * p + a] = w[a];
            double xa = Xc[a] + v[a];
            if (fixed_p) {
                xa = Xc[a];
            } else if (per[a]) {
                if (xa >= box[a]) xa -= box[a];
                else if (xa < 0.0) xa += box[a];
            } else {
                if (xa < 0.0 || xa > box[a] - 1.0) atomicOr(s.flags, 0x10u);
                xa = fmin(fmax(xa, 0.0), box[a] - 1.0);
            }
            Xn[3 * p + a] = xa;
        }
        // the fluid kernel's wall state of this step: X(t) and the new velocities
        pack_state(s.pf[par] + 12 * p, Xo + 3 * p, v, w);
    }
}


// ---------------------------------------------------------------------------
// re-projection kernel
// ---------------------------------------------------------------------------
// Per-particle context of the re-projection: the particle, its lattice, its position
// after this step's motion (mode 0) or now (mode 1), and its near neighbours (staged in
// the workgroup's shared memory, slot w).
struct RemapCtx {
    int p, w, nn;
    const MemberDev *M;
    double X[3], R, R2;
    int per[3];
    double box[3];
};

constexpr int kRemapWaves = 4; // particles per workgroup of the re-projection kernel

// Re-projection (Sec. 2.3), one wave per particle for the common case: the candidates of
// a small step, from the particle's surface band or shell list, evaluated by the wave's
// 64 lanes.  A particle that needs its shell list rebuilt (set-up, or motion beyond the
// shell) and the periodic near-list build use the whole workgroup, one particle after the
// other.  Workgroups past the particles reduce the probe planes.
template <int P>
__global__ __launch_bounds__(256) void k_remap(DevSet s, int mode, int only)
{
    using S = typename Prec<P>::S;
    __shared__ double red[4][8];
    __shared__ double nbw[kRemapWaves][kNearCap][4];
    __shared__ int nbidw[kRemapWaves][kNearCap];
    __shared__ int cnt4[4];
    __shared__ int cstart[kChunks + 1];
    __shared__ double accw[kRemapWaves][6];
    __shared__ double ctxw[kRemapWaves][9]; // x, x_ref unwrapped next to x, lr, dr, overlap depth
    __shared__ int flagw[kRemapWaves];
    __shared__ int ncnt[kRemapWaves][4]; // near-list candidates per (particle, wave)
    // each wave's queue of candidate nodes (cell, owner before the projection or -2)
    constexpr int kQueue = 256;
    __shared__ int qcell[kRemapWaves][kQueue], qwas[kRemapWaves][kQueue];
    // the step being completed: copied by the fluid kernel (mode 0); the counter itself is
    // advanced here and read by no workgroup of this kernel
    const long long t = (mode == 0) ? *s.tcopy : *s.tstep;
    const int par = (int)(t & 1);
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int npw = (s.ptot + kRemapWaves - 1) / kRemapWaves;
    if (mode == 0 && blockIdx.x == 0 && tid == 0) *s.tstep = t + 1;

    if ((int)blockIdx.x >= npw) {
        // probe plane reduction, one workgroup per (lattice, probe), tiles in fixed order
        if (mode != 0) return;
        const int q = blockIdx.x - npw;
        if (q >= s.nprobe_total) return;
        int m = 0;
        while (m + 1 < s.nmem && s.mem[m + 1].plist_off <= q) ++m;
        while (s.mem[m].n_probe == 0 || q - s.mem[m].plist_off >= s.mem[m].n_probe) ++m;
        const MemberDev *Mq = s.mem + m;
        const int k = q - Mq->plist_off;
        const int z = s.plist[Mq->plist_off + k];
        const int tz = z / s.nzt, dz = z - tz * s.nzt;
        const int ntile = Mq->ntx * Mq->nty;
        double v[4] = {0, 0, 0, 0};
        for (int c = tid; c < ntile; c += 256) {
            const long long gt = Mq->tile_off + (long long)tz * ntile + c;
            const double *pp = s.pprt + (gt * s.nzt + dz) * 4;
            v[0] += pp[0]; v[1] += pp[1]; v[2] += pp[2]; v[3] += pp[3];
        }
        block_sum<4>(v, red);
        if (tid == 0) {
            double *o = s.ring + Mq->ring_off + ((t % s.ring_len) * Mq->n_probe + k) * 4;
            o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
        }
        return;
    }

    const int sp = (mode == 1) ? par : (par ^ 1); // buffers of the positions after the motion
    const double *Xs = s.X[sp], *Vs = s.V[sp], *Ws = s.W[sp];
    const int sn = par ^ 1;                       // population buffer holding f~(t+1)

    auto dist2c = [&](const RemapCtx &c, int i, int j, int k, double X0, double X1, double X2) {
        const double dx = mimg((double)i - X0, c.per[0], c.box[0]);
        const double dy = mimg((double)j - X1, c.per[1], c.box[1]);
        const double dz = mimg((double)k - X2, c.per[2], c.box[2]);
        return (dx * dx + dy * dy) + dz * dz;
    };

    // owner of one node after the motion; conversions of covered / uncovered nodes
    auto evaluate = [&](const RemapCtx &c, int ii, int jj, int kk, int cell, double d2n, int was_pre,
                        double (&acc)[6], int &conv) {
        const MemberDev *M = c.M;
        const int p = c.p;
        const int dims[3] = {M->nx, M->ny, M->nz};
        const int *cur = s.own[par] + M->cell_off;
        // owner: smallest d^2, then smallest index, among the spheres containing the node
        int best = -1;
        double bd = 0.0;
        if (d2n <= c.R2) { best = p; bd = d2n; }
        for (int k = 0; k < c.nn; ++k) {
            const double dq = dist2c(c, ii, jj, kk, nbw[c.w][k][0], nbw[c.w][k][1], nbw[c.w][k][2]);
            if (dq <= nbw[c.w][k][3] * nbw[c.w][k][3]) {
                const int q = nbidw[c.w][k];
                if (best < 0 || dq < bd || (dq == bd && q < best)) { best = q; bd = dq; }
            }
        }
        if (mode == 1) {
            if (best >= 0) { s.own[0][M->cell_off + cell] = best; s.own[1][M->cell_off + cell] = best; }
            return;
        }
        const int was = (was_pre >= -1) ? was_pre : cur[cell];
        if (best == was) return;
        s.own[par ^ 1][M->cell_off + cell] = best;
        // the 18 neighbours and their owners before the re-projection (loads together)
        int nbc[kQ - 1], ow[kQ - 1];
#pragma unroll
        for (int e = 0; e < kQ - 1; ++e) {
            int cc[3] = {ii + kCX[e], jj + kCY[e], kk + kCZ[e]};
            bool ok = true;
            for (int a = 0; a < 3; ++a) {
                if (cc[a] < 0 || cc[a] >= dims[a]) {
                    if (c.per[a]) cc[a] = cc[a] < 0 ? cc[a] + dims[a] : cc[a] - dims[a];
                    else ok = false;
                }
            }
            nbc[e] = ok ? (cc[2] * dims[1] + cc[1]) * dims[0] + cc[0] : -1;
        }
#pragma unroll
        for (int e = 0; e < kQ - 1; ++e) ow[e] = nbc[e] >= 0 ? cur[nbc[e]] : -1;
        // (the cached link entries that this change makes stale are marked by the next
        // refresh, which sees which link words actually change)
        const int slot = atomicAdd(s.chgcnt + par, 1);
        if (slot < s.chg_cap) {
            s.chg[par][2 * slot] = (int)(M->cell_off + cell);
            s.chg[par][2 * slot + 1] = best;
        } else {
            atomicOr(s.flags, 0x4u);
        }
        const double r0 = mimg((double)ii - c.X[0], c.per[0], c.box[0]);
        const double r1 = mimg((double)jj - c.X[1], c.per[1], c.box[1]);
        const double r2 = mimg((double)kk - c.X[2], c.per[2], c.box[2]);
        S *Bn = (S *)(sn ? s.popB : s.popA) + M->pop_off;
        const int nc = (int)M->ncell;
        const double rho_ff = M->rho_f;
        if (was < 0 && best == p) {
            // Eq. (convertFS): a covered node hands its momentum to the particle
            const int sl = node_slot(s, M, cell, ii, jj, kk);
            if (sl < 0) { atomicOr(s.flags, 0x100u); return; }
            double f[kQ];
#pragma unroll
            for (int d = 0; d < kQ; ++d) f[d] = (double)ld<P>(Bn, d * nc + sl, d, rho_ff);
            double rho, j0, j1, j2;
            moments<double>(f, rho, j0, j1, j2);
            conv = 1;
            acc[0] += j0; acc[1] += j1; acc[2] += j2;
            acc[3] += r1 * j2 - r2 * j1;
            acc[4] += r2 * j0 - r0 * j2;
            acc[5] += r0 * j1 - r1 * j0;
        } else if (was == p && best < 0) {
            // Eq. (convertSF): an uncovered node is refilled with f^eq(rho_bar, V_b)
            // and takes rho_bar V_b from the particle; rho_bar averages the
            // neighbours that are fluid before and after the re-projection.  Under
            // compact storage a node outside the lists has its refill parked for the
            // list rebuild at the start of the next step.
            unsigned use = 0u;
#pragma unroll
            for (int e = 0; e < kQ - 1; ++e) {
                if (nbc[e] < 0 || ow[e] >= 0) continue;
                const int yc = nbc[e];
                const int zc = yc / (dims[0] * dims[1]), rc = yc - zc * dims[0] * dims[1];
                const int yy = rc / dims[0], xx = rc - yy * dims[0];
                bool inside = dist2c(c, xx, yy, zc, c.X[0], c.X[1], c.X[2]) <= c.R2;
                for (int k = 0; k < c.nn && !inside; ++k)
                    inside = dist2c(c, xx, yy, zc, nbw[c.w][k][0], nbw[c.w][k][1], nbw[c.w][k][2]) <=
                             nbw[c.w][k][3] * nbw[c.w][k][3];
                if (!inside) use |= 1u << e;
            }
            const int sl = node_slot(s, M, cell, ii, jj, kk);
            double sum = 0.0;
            int cnt = 0;
#pragma unroll 1
            for (int e = 0; e < kQ - 1; ++e) {
                if (!((use >> e) & 1u)) continue;
                int yc = 0;
#pragma unroll
                for (int q = 0; q < kQ - 1; ++q)
                    if (q == e) yc = nbc[q];
                if (s.compact) {
                    const int zc = yc / (dims[0] * dims[1]), rc = yc - zc * dims[0] * dims[1];
                    const int yy = rc / dims[0];
                    yc = slot_of(s, M, rc - yy * dims[0], yy, zc);
                    if (yc < 0) { atomicOr(s.flags, 0x100u); continue; }
                }
                double rr = 0.0;
                for (int d = 0; d < kQ; ++d) rr += (double)ld<P>(Bn, d * nc + yc, d, rho_ff);
                sum += rr;
                cnt += 1;
            }
            const double rbar = cnt > 0 ? sum / cnt : M->rho_f;
            const double *Vp = Vs + 3 * p, *Wp = Ws + 3 * p;
            const double vb0 = Vp[0] + (Wp[1] * r2 - Wp[2] * r1);
            const double vb1 = Vp[1] + (Wp[2] * r0 - Wp[0] * r2);
            const double vb2 = Vp[2] + (Wp[0] * r1 - Wp[1] * r0);
            const double uu = vb0 * vb0 + vb1 * vb1 + vb2 * vb2;
            if (sl >= 0) {
#pragma unroll
                for (int d = 0; d < kQ; ++d)
                    st<P>(Bn, d * nc + sl, d, (typename Prec<P>::C)feq<double>(d, rbar, vb0, vb1, vb2, uu), rho_ff);
            } else {
                const int pi = atomicAdd(s.pcnt + par, 1);
                if (pi < kPendCap) {
                    double *rec = s.pbuf[par] + 4 * pi;
                    rec[0] = rbar; rec[1] = vb0; rec[2] = vb1; rec[3] = vb2;
                    s.pend[M->cell_off + cell] = pi;
                    *s.relist_at = t + 1;
                    atomicOr(s.flags, 0x200u);
                } else {
                    atomicOr(s.flags, 0x100u);
                }
            }
            conv = 1;
            const double m0 = rbar * vb0, m1 = rbar * vb1, m2 = rbar * vb2;
            acc[0] -= m0; acc[1] -= m1; acc[2] -= m2;
            acc[3] -= r1 * m2 - r2 * m1;
            acc[4] -= r2 * m0 - r0 * m2;
            acc[5] -= r0 * m1 - r1 * m0;
        }
    };

    // ------------------------------------------------------------------------------
    // phase A: one wave per particle
    // ------------------------------------------------------------------------------
    const int p = blockIdx.x * kRemapWaves + wv;
    // Per-particle values that depend on nothing else are loaded together, before any
    // branch (index clamped past the particles): the member, the near list, the reference
    // state, the first band entries of each lane, and p's position in both buffers.
    constexpr int kPre = 4; // band entries preloaded per lane
    bool active = p < s.ptot;
    const int pc = active ? p : 0;
    const int m = s.pmem[pc];
    const int nn_raw = s.nnear[pc];
    const int q_raw = s.nearl[(long long)pc * kNearCap + (lane & (kNearCap - 1))];
    const double Rp = s.R[pc];
    const double Xr_ld[3] = {s.Xref[3 * pc], s.Xref[3 * pc + 1], s.Xref[3 * pc + 2]};
    const double Xb0[3] = {s.X[0][3 * pc], s.X[0][3 * pc + 1], s.X[0][3 * pc + 2]};
    const double Xb1[3] = {s.X[1][3 * pc], s.X[1][3 * pc + 1], s.X[1][3 * pc + 2]};
    const double Xl_ld[3] = {s.Xl[3 * pc], s.Xl[3 * pc + 1], s.Xl[3 * pc + 2]};
    const double mg_ld = s.margin[pc], rdisp_ld = s.rdisp[pc], rlens_ld = s.rlens[pc];
    const long long nat_ld = s.near_at[pc];
    const int bnum = min(s.bcnt[pc], s.bcap);
    int bc[kPre];
    float bd[kPre];
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
        const int k = lane + 64 * i;
        // (every lane loads: past the band's end it reads the first entry)
        const int kc = (k < bnum) ? k : 0;
        const int bcr = s.bcell[(long long)pc * s.bcap + kc];
        const float bdr = s.bdr[(long long)pc * s.bcap + kc];
        bc[i] = (k < bnum) ? bcr : 0;
        bd[i] = (k < bnum) ? bdr : 0.0f;
    }
    const MemberDev *Mp = nullptr;
    if (active) {
        Mp = s.mem + m;
        active = (p - Mp->p_off < Mp->np) && (only < 0 || m == only);
    }
    int flag = 0; // 1 active, 2 shell rebuild, 4 near-list build
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int conv = 0;
    if (active) {
        RemapCtx c;
        c.p = p; c.w = wv; c.M = Mp;
        for (int a = 0; a < 3; ++a) {
            c.per[a] = Mp->per[a];
            c.box[a] = Mp->box[a];
            c.X[a] = sp ? Xb1[a] : Xb0[a];
        }
        c.R = Rp; c.R2 = Rp * Rp;
        c.nn = min(nn_raw, kNearCap);
        const double Xr[3] = {mode == 1 ? c.X[0] : Xr_ld[0], mode == 1 ? c.X[1] : Xr_ld[1], mode == 1 ? c.X[2] : Xr_ld[2]};
        if (lane < c.nn) {
            const int q = q_raw;
            nbidw[wv][lane] = q;
            nbw[wv][lane][0] = Xs[3 * q]; nbw[wv][lane][1] = Xs[3 * q + 1]; nbw[wv][lane][2] = Xs[3 * q + 2];
            nbw[wv][lane][3] = s.R[q];
        }
        // owners of the preloaded band entries (the candidates of a small step)
        const int *cur = s.own[par] + Mp->cell_off;
        int was[kPre];
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
            const int wr = cur[bc[i]];
            was[i] = (lane + 64 * i < bnum) ? wr : -1;
        }
        // the wave's staged neighbours are visible to all its lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // overlap depth with the near neighbours (one lane each), maximum over the wave
        double dmax = 0.0;
        if (lane < c.nn) {
            const double d0 = mimg(nbw[wv][lane][0] - c.X[0], c.per[0], c.box[0]);
            const double d1 = mimg(nbw[wv][lane][1] - c.X[1], c.per[1], c.box[1]);
            const double d2 = mimg(nbw[wv][lane][2] - c.X[2], c.per[2], c.box[2]);
            dmax = fmax(0.0, c.R + nbw[wv][lane][3] - sqrt((d0 * d0 + d1 * d1) + d2 * d2));
        }
        for (int off = 32; off >= 1; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
        double disp2 = 0.0, xr[3];
        for (int a = 0; a < 3; ++a) {
            const double d = mimg(c.X[a] - Xr[a], c.per[a], c.box[a]);
            disp2 += d * d;
            xr[a] = c.X[a] - d; // reference centre unwrapped next to X
        }
        // node lists: rebuilt at the start of the next step once p may have moved the skin
        if (s.listmode) {
            if (mode == 1) {
                if (lane == 0) {
                    *s.relist_at = t;
                    const double *Vp = Vs + 3 * p;
                    s.pspd[p] = sqrt(Vp[0] * Vp[0] + Vp[1] * Vp[1] + Vp[2] * Vp[2]);
                }
            } else {
                double dl = 0.0, ds = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double d = mimg(c.X[a] - Xl_ld[a], c.per[a], c.box[a]);
                    const double v = mimg(c.X[a] - (sp ? Xb0[a] : Xb1[a]), c.per[a], c.box[a]);
                    dl += d * d;
                    ds += v * v;
                }
                // a node uncovered by the next re-projection should have a slot in the
                // current lists, so they are rebuilt while the particle stays within the
                // skin after one more step of up to list_margin times this step's
                // displacement (under compact storage a node uncovered outside them is
                // parked until the rebuild)
                const double reach = sqrt(dl) + s.list_margin * sqrt(ds);
                if (lane == 0) {
                    s.pspd[p] = sqrt(ds);
                    if (reach >= s.skin[m] - 1e-9) *s.relist_at = t + 1;
                }
            }
        }
        // Candidates, with d_ref = |x - X_ref| and maxima over this projection and every
        // one since the shell list was built at X_ref (the node map being replaced comes
        // from the previous one): a node enters or leaves p only if |d_ref - R| <= dr,
        // dr = max |X - X_ref|; the order between p and an overlapping sphere changes only
        // at nodes inside p within the overlap depth, d_ref - R >= -lr, lr = max(|X -
        // X_ref| + overlap depth).  A node with d_ref - R > dr is outside p at both
        // projections, so its owner is settled by the other spheres' workgroups.
        const double disp = sqrt(disp2);
        const double rd = (mode == 1) ? disp : fmax(rdisp_ld, disp);
        const double rl = (mode == 1) ? disp + dmax : fmax(rlens_ld, disp + dmax);
        const double dr = rd + 1e-9, lr = rl + 1e-9;
        // the shell list around X_ref holds every node with |d_ref - R| < kShell: while
        // lr stays below kShell the candidates are in it, else it is rebuilt at X
        const bool rebuild = (mode == 1) || (lr >= kShell - 1e-6);
        const bool use_list = !rebuild && (lr >= mg_ld);
        if (use_list) {
            // candidates have -lr <= d_ref - R <= dr: the band list holds them all while
            // lr <= kBandIn and dr <= kBandOut, the whole shell list otherwise
            const bool band = lr + 1e-6 <= kBandIn && dr + 1e-6 <= kBandOut;
            const long long lbase = (long long)p * s.lcap;
            const int n = band ? bnum : s.lcnt[p];
            const int *lc = band ? s.bcell + (long long)p * s.bcap : s.lcell + lbase;
            const float *dl = band ? s.bdr + (long long)p * s.bcap : s.ldr + lbase;
            const int dxy = Mp->nx * Mp->ny, dx = Mp->nx;
            static_assert(64 * kPre == kQueue, "one queue slot per entry of a batch");
            const unsigned long long below = (1ull << lane) - 1ull;
            // kPre entries per lane at a time (the first batch of the band is loaded
            // already): the ones within the candidate range go to the wave's queue in list
            // order, and the queue is evaluated 64 nodes at a time, so a wave evaluates
            // ceil(candidates / 64) rounds per batch instead of one round per entry round
            for (int base = 0; base < n; base += kQueue) {
                int qn = 0;
#pragma unroll
                for (int u = 0; u < kPre; ++u) {
                    const int k = base + 64 * u + lane;
                    int cell = 0, wpre = -2;
                    double dk = 0.0;
                    if (band && base == 0) {
                        cell = bc[u]; dk = (double)bd[u]; wpre = was[u];
                    } else if (k < n) {
                        cell = lc[k]; dk = (double)dl[k];
                    }
                    const bool take = k < n && !(dk < -lr - 1e-6 || dk > dr + 1e-6);
                    const unsigned long long bal = __ballot(take);
                    if (take) {
                        const int at = qn + __popcll(bal & below);
                        qcell[wv][at] = cell;
                        qwas[wv][at] = wpre;
                    }
                    qn += __popcll(bal);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int q = lane; q < qn; q += 64) {
                    const int cell = qcell[wv][q], wpre = qwas[wv][q];
                    const int kk = cell / dxy;
                    const int rem = cell - kk * dxy;
                    const int jj = rem / dx, ii = rem - jj * dx;
                    evaluate(c, ii, jj, kk, cell, dist2c(c, ii, jj, kk, c.X[0], c.X[1], c.X[2]), wpre, acc, conv);
                }
                // (the next batch refills the queue once every lane has read its entry)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        flag = 1 | (rebuild ? 2 : 0) | ((mode == 0 && t + 1 - nat_ld >= kNearEvery) ? 4 : 0);
        if (lane == 0) {
            ctxw[wv][0] = c.X[0]; ctxw[wv][1] = c.X[1]; ctxw[wv][2] = c.X[2];
            ctxw[wv][3] = xr[0]; ctxw[wv][4] = xr[1]; ctxw[wv][5] = xr[2];
            ctxw[wv][6] = lr; ctxw[wv][7] = dr; ctxw[wv][8] = dmax;
            if (mode == 0 && !rebuild) {
                s.rdisp[p] = rd;
                s.rlens[p] = rl;
            }
        }
    }
    // the wave's conversion momentum (summed only when a lane made a conversion)
    if (__ballot(conv) != 0ull) {
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] = wave_sum(acc[k]);
    }
    if (lane == 0) {
        flagw[wv] = flag;
        for (int k = 0; k < 6; ++k) accw[wv][k] = acc[k];
    }
    __syncthreads();

    // ------------------------------------------------------------------------------
    // phase B: shell-list rebuilds and near-list builds, the whole workgroup per particle
    // ------------------------------------------------------------------------------
    // (the near lists of the workgroup's particles are built in one pass over the
    // candidates when those particles share a lattice, which is the rule)
    int near_w = 0, near_m = -1;
    bool near_joint = true;
    for (int w = 0; w < kRemapWaves; ++w) {
        if (!(flagw[w] & 4)) continue;
        const int mw = s.pmem[blockIdx.x * kRemapWaves + w];
        near_joint = near_joint && (near_m < 0 || mw == near_m);
        near_m = mw;
        near_w |= 1 << w;
    }
    for (int w = 0; w < kRemapWaves; ++w) {
        const int fw = flagw[w] & (near_joint ? 3 : 7);
        if ((fw & 6) == 0) continue;
        const int pw = blockIdx.x * kRemapWaves + w;
        RemapCtx c;
        c.p = pw; c.w = w; c.M = s.mem + s.pmem[pw];
        const MemberDev *M = c.M;
        for (int a = 0; a < 3; ++a) {
            c.per[a] = M->per[a];
            c.box[a] = M->box[a];
            c.X[a] = ctxw[w][a];
        }
        c.R = s.R[pw]; c.R2 = c.R * c.R;
        c.nn = min(s.nnear[pw], kNearCap);
        const double xr[3] = {ctxw[w][3], ctxw[w][4], ctxw[w][5]};
        const double lr = ctxw[w][6], dr = ctxw[w][7], dmax = ctxw[w][8];
        const double R = c.R, R2 = c.R2;
        const int dims[3] = {M->nx, M->ny, M->nz};
        const double Xr[3] = {mode == 1 ? c.X[0] : s.Xref[3 * pw], mode == 1 ? c.X[1] : s.Xref[3 * pw + 1],
                              mode == 1 ? c.X[2] : s.Xref[3 * pw + 2]};
        if (fw & 2) {
            double acc2[6] = {0, 0, 0, 0, 0, 0};
            int conv2 = 0;
            // scan the boxes around X and X_ref, evaluate the candidates, and rebuild the
            // shell list at X: nodes with -kShell < d - R <= sqrt(2) + kShell, with the
            // directions e whose source x - c_e lies within R + kShell (link candidates)
            const double hout = R + 1.5 + kShell + lr;
            const double Rin = R - kShell, Rin2 = Rin > 0.0 ? Rin * Rin : -1.0, Rout2 = hout * hout;
            const double Rl2 = (R + kShell) * (R + kShell);
            const long long lbase = (long long)pw * s.lcap;
            int lo[3], ext[3];
            for (int a = 0; a < 3; ++a) {
                int l = (int)floor(fmin(c.X[a], xr[a]) - hout) - 1;
                int h = (int)ceil(fmax(c.X[a], xr[a]) + hout) + 1;
                if (!c.per[a]) { l = max(l, 0); h = min(h, dims[a] - 1); }
                else if (h - l + 1 > dims[a]) { l = 0; h = dims[a] - 1; } // visit each node once
                lo[a] = l;
                ext[a] = max(h - l + 1, 0);
            }
            const int tot = ext[0] * ext[1] * ext[2];
            double mrg = kShell;
            int lcount = 0, bcount = 0;
            const long long bbase = (long long)pw * s.bcap;
            // chunks of the list are z-slabs of hz planes of the scan box
            const int hz = (ext[2] + kChunks - 1) / kChunks;
            if (tid <= kChunks) cstart[tid] = 0;
            __syncthreads();
            for (int base = 0; base < tot; base += 256) {
                const int idx = base + tid;
                bool in_list = false;
                int cell = 0;
                unsigned mask = 0u;
                float dref = 0.0f;
                if (idx < tot) {
                    int ii = lo[0] + idx % ext[0];
                    int jj = lo[1] + (idx / ext[0]) % ext[1];
                    int kk = lo[2] + idx / (ext[0] * ext[1]);
                    // (positions stay within one period of the lattice, so one wrap suffices;
                    // a true modulo keeps every index in range regardless)
                    ii = ((ii % dims[0]) + dims[0]) % dims[0];
                    jj = ((jj % dims[1]) + dims[1]) % dims[1];
                    kk = ((kk % dims[2]) + dims[2]) % dims[2];
                    cell = (kk * dims[1] + jj) * dims[0] + ii;
                    const double d2n = dist2c(c, ii, jj, kk, c.X[0], c.X[1], c.X[2]);
                    bool ev;
                    if (mode == 1) {
                        ev = d2n <= R2;
                    } else {
                        const double dd = sqrt(dist2c(c, ii, jj, kk, Xr[0], Xr[1], Xr[2])) - R;
                        ev = dd >= -lr && dd <= dr;
                    }
                    if (ev) evaluate(c, ii, jj, kk, cell, d2n, -2, acc2, conv2);
                    if (d2n > Rin2 && d2n <= Rout2) {
                        const double dn = sqrt(d2n) - R;
                        if (dn > -kShell && dn <= 1.4142135623730951 + kShell) {
                            in_list = true;
                            dref = (float)dn;
                            mrg = fmin(mrg, fabs(dn));
#pragma unroll
                            for (int e = 0; e < kQ - 1; ++e) {
                                const int si = ii - kCX[e], sj = jj - kCY[e], sk = kk - kCZ[e];
                                if ((!c.per[0] && (si < 0 || si >= dims[0])) || (!c.per[1] && (sj < 0 || sj >= dims[1])) ||
                                    (!c.per[2] && (sk < 0 || sk >= dims[2])))
                                    continue;
                                if (dist2c(c, wrapc(si, dims[0]), wrapc(sj, dims[1]), wrapc(sk, dims[2]), c.X[0], c.X[1],
                                           c.X[2]) <= Rl2)
                                    mask |= 1u << e;
                            }
                        }
                    }
                }
                int tcount = 0;
                const int rk = block_rank(in_list, tcount, cnt4);
                if (in_list && hz > 0) atomicAdd(&cstart[idx / (ext[0] * ext[1]) / hz + 1], 1);
                if (in_list) {
                    const int slot = lcount + rk;
                    if (slot < s.lcap) {
                        s.lcell[lbase + slot] = cell;
                        s.ldr[lbase + slot] = dref;
                        s.lmask[lbase + slot] = mask;
                    } else {
                        atomicOr(s.flags, 0x40u);
                    }
                }
                lcount += tcount;
                // the surface band, a sub-list for small displacements
                const bool in_band = in_list && (double)dref >= -kBandIn && (double)dref <= kBandOut;
                const int bk = block_rank(in_band, tcount, cnt4);
                if (in_band) {
                    const int slot = bcount + bk;
                    if (slot < s.bcap) {
                        s.bcell[bbase + slot] = cell;
                        s.bdr[bbase + slot] = dref;
                    } else {
                        atomicOr(s.flags, 0x40u);
                    }
                }
                bcount += tcount;
            }
            double mv = wave_min_d(mrg);
            if ((tid & 63) == 0) red[tid >> 6][7] = mv;
            __syncthreads();
            if (tid == 0) {
                mv = fmin(fmin(red[0][7], red[1][7]), fmin(red[2][7], red[3][7]));
                s.margin[pw] = mv;
                s.lcnt[pw] = min(lcount, s.lcap);
                s.bcnt[pw] = min(bcount, s.bcap);
                s.lreb[pw] = (mode == 1) ? t - 1 : t; // the next link pass recomputes its links
                s.lzr[2 * pw] = lo[2];
                s.lzr[2 * pw + 1] = hz;
                int acc_c = 0;
                for (int k = 0; k <= kChunks; ++k) {
                    acc_c += cstart[k];
                    s.lchunk[pw * (kChunks + 1) + k] = min(acc_c, s.lcap);
                }
                s.Xref[3 * pw] = c.X[0]; s.Xref[3 * pw + 1] = c.X[1]; s.Xref[3 * pw + 2] = c.X[2];
                // maxima restart at the new reference, where this projection has
                // displacement 0 and overlap depth dmax
                s.rdisp[pw] = 0.0;
                s.rlens[pw] = dmax;
            }
            // the momentum of this rebuild's conversions
            if (mode == 0 && __syncthreads_or(conv2)) {
                block_sum<6>(acc2, red);
                if (tid == 0)
                    for (int k = 0; k < 6; ++k) accw[w][k] += acc2[k];
            }
            __syncthreads();
        }
        if (fw & 4) {
            // the near list for the next kNearEvery steps, from the positions after this
            // step's motion: every particle within R_p + R_q + kNearMargin (each particle
            // moves less than 0.25 per step, so the contacts and the spheres that can own
            // a node of p stay among them until the next build)
            const int q0 = M->p_off, nq = M->np;
            int near_total = 0;
            for (int base = 0; base < nq; base += 256) {
                const int jj = base + tid;
                bool isnear = false;
                if (jj < nq && q0 + jj != pw) {
                    const int q = q0 + jj;
                    const double d0 = mimg(Xs[3 * q] - c.X[0], c.per[0], c.box[0]);
                    const double d1 = mimg(Xs[3 * q + 1] - c.X[1], c.per[1], c.box[1]);
                    const double d2 = mimg(Xs[3 * q + 2] - c.X[2], c.per[2], c.box[2]);
                    isnear = sqrt((d0 * d0 + d1 * d1) + d2 * d2) <= R + s.R[q] + kNearMargin;
                }
                int tot = 0;
                const int rk = block_rank(isnear, tot, cnt4);
                if (isnear) {
                    const int slot = near_total + rk;
                    if (slot < kNearCap) s.nearl[(long long)pw * kNearCap + slot] = q0 + jj;
                    else atomicOr(s.flags, 0x2u);
                }
                near_total += tot;
            }
            if (tid == 0) {
                s.nnear[pw] = min(near_total, kNearCap);
                s.near_at[pw] = t + 1;
            }
            __syncthreads();
        }
    }
    if (near_joint && near_w != 0) {
        // the same near lists for the particles of the workgroup together: each candidate's
        // position is loaded once and tested against every one of them
        const MemberDev *M = s.mem + near_m;
        const int q0 = M->p_off, nq = M->np;
        const int per[3] = {M->per[0], M->per[1], M->per[2]};
        const double box[3] = {M->box[0], M->box[1], M->box[2]};
        double Rw[kRemapWaves];
#pragma unroll
        for (int w = 0; w < kRemapWaves; ++w) Rw[w] = s.R[min((int)blockIdx.x * kRemapWaves + w, s.ptot - 1)];
        int near_total[kRemapWaves] = {};
        const unsigned long long below = (1ull << (tid & 63)) - 1ull;
        for (int base = 0; base < nq; base += 256) {
            const int jj = base + tid;
            const int q = q0 + min(jj, nq - 1);
            const double Y0 = Xs[3 * q], Y1 = Xs[3 * q + 1], Y2 = Xs[3 * q + 2], Rq = s.R[q];
            // the candidate's verdict for every particle of the workgroup, then one exchange
            // of the waves' counts ranks the candidates of all of them in thread order
            bool isnear[kRemapWaves];
            unsigned long long bal[kRemapWaves];
#pragma unroll
            for (int w = 0; w < kRemapWaves; ++w) {
                const int pw = blockIdx.x * kRemapWaves + w;
                isnear[w] = false;
                if (((near_w >> w) & 1) && jj < nq && q != pw) {
                    const double d0 = mimg(Y0 - ctxw[w][0], per[0], box[0]);
                    const double d1 = mimg(Y1 - ctxw[w][1], per[1], box[1]);
                    const double d2 = mimg(Y2 - ctxw[w][2], per[2], box[2]);
                    isnear[w] = sqrt((d0 * d0 + d1 * d1) + d2 * d2) <= Rw[w] + Rq + kNearMargin;
                }
                bal[w] = __ballot(isnear[w]);
                if ((tid & 63) == 0) ncnt[w][wv] = __popcll(bal[w]);
            }
            __syncthreads();
#pragma unroll
            for (int w = 0; w < kRemapWaves; ++w) {
                int off = 0, tot = 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = ncnt[w][v];
                    off += (v < wv) ? c : 0;
                    tot += c;
                }
                if (isnear[w]) {
                    const int slot = near_total[w] + off + __popcll(bal[w] & below);
                    const int pw = blockIdx.x * kRemapWaves + w;
                    if (slot < kNearCap) s.nearl[(long long)pw * kNearCap + slot] = q;
                    else atomicOr(s.flags, 0x2u);
                }
                near_total[w] += tot;
            }
            __syncthreads();
        }
#pragma unroll
        for (int w = 0; w < kRemapWaves; ++w) {
            if (tid == w && ((near_w >> w) & 1)) {
                const int pw = blockIdx.x * kRemapWaves + w;
                s.nnear[pw] = min(near_total[w], kNearCap);
                s.near_at[pw] = t + 1;
            }
        }
    }
    // the conversion momentum of each particle of the workgroup
    if (mode == 0 && tid < kRemapWaves && (flagw[tid] & 1)) {
        const int pw = blockIdx.x * kRemapWaves + tid;
        for (int a = 0; a < 3; ++a) { s.Ph[3 * pw + a] = accw[tid][a]; s.Lh[3 * pw + a] = accw[tid][3 + a]; }
    }
}

// ---------------------------------------------------------------------------
// initial populations f = w_d rho_f in both buffers
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_init_pops(DevSet s, long long total_cells)
{
    using S = typename Prec<P>::S;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total_cells) return;
    const MemberDev *M = member_of_cell(s, c);
    const int cell = (int)(c - M->cell_off);
    const int nc = (int)M->ncell;
    S *A = (S *)s.popA + M->pop_off, *B = (S *)s.popB + M->pop_off;
    const double rho_ff = M->rho_f;
    for (int d = 0; d < kQ; ++d) {
        const typename Prec<P>::C v = (typename Prec<P>::C)(kWd[d] * M->rho_f);
        st<P>(A, d * nc + cell, d, v, rho_ff);
        st<P>(B, d * nc + cell, d, v, rho_ff);
    }
}

// ---------------------------------------------------------------------------
// macroscopic fields of one lattice (node layout): rho = sum_d f_d, rho u = sum_d f_d c_d
// (Eq. rhoAndU) in FP64, directions in index order; 0 at solid nodes.  out: [4][ncell]
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_fields(DevSet s, int m, double *out)
{
    const long long t = *s.tstep;
    const int par = (int)(t & 1);
    const MemberDev *M = s.mem + m;
    const long long nc = M->ncell;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    using S = typename Prec<P>::S;
    const S *A = (const S *)(par ? s.popB : s.popA) + M->pop_off;
    double rho = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    if (s.own[par][M->cell_off + c] < 0) {
        const double rho_ff = M->rho_f;
        for (int d = 0; d < kQ; ++d) {
            const double f = (double)ld<P>(A, (unsigned)(d * nc + c), d, rho_ff);
            rho += f;
            j0 += f * kCXd[d];
            j1 += f * kCYd[d];
            j2 += f * kCZd[d];
        }
        j0 /= rho; j1 /= rho; j2 /= rho;
    }
    out[c] = rho;
    out[nc + c] = j0;
    out[2 * nc + c] = j1;
    out[3 * nc + c] = j2;
}

// ---------------------------------------------------------------------------
// compact storage back to the node layout (before the host reads or writes populations,
// or replaces particles): per plane, listed nodes move from their slots to their nodes,
// every other node takes the rest state w_d rho_f, and the row tables become the identity
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_expand(DevSet s)
{
    using S = typename Prec<P>::S;
    const long long t = *s.tstep;
    const int par = (int)(t & 1);
    for (int pl = blockIdx.x; pl < s.nplanes; pl += gridDim.x) {
        int lo = 0, hi = s.nmem - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s.mem[mid].pz_off <= pl) lo = mid;
            else hi = mid - 1;
        }
        const MemberDev *M = s.mem + lo;
        const int z = pl - M->pz_off, nx = M->nx, ny = M->ny, nxy = nx * ny, nw = M->nw;
        const long long nc = M->ncell;
        S *A = (S *)(par ? s.popB : s.popA) + M->pop_off;
        S *Cb = (S *)s.popC + M->pop_off;
        const double rho_ff = M->rho_f;
        const long long z0 = (long long)z * nxy;
        // the list of this plane is the one the row tables were built from
        for (int c = threadIdx.x; c < nxy; c += blockDim.x) {
            const int j = c / nx, i = c - j * nx;
            const int sl = slot_of(s, M, i, j, z);
            if (sl >= 0)
                for (int d = 0; d < kQ; ++d) Cb[d * nc + z0 + c] = A[d * nc + sl];
        }
        __threadfence_block();
        __syncthreads();
        for (int c = threadIdx.x; c < nxy; c += blockDim.x) {
            const int j = c / nx, i = c - j * nx;
            if (slot_of(s, M, i, j, z) >= 0) {
                for (int d = 0; d < kQ; ++d) A[d * nc + z0 + c] = Cb[d * nc + z0 + c];
            } else {
                // a parked refill of the last re-projection, else the rest state
                const long long gcell = M->cell_off + z0 + c;
                const int pi = s.pend[gcell];
                double rb = M->rho_f, u0 = 0.0, u1 = 0.0, u2 = 0.0;
                if (pi >= 0) {
                    const double *rec = s.pbuf[par ^ 1] + 4 * pi;
                    rb = rec[0]; u0 = rec[1]; u1 = rec[2]; u2 = rec[3];
                    s.pend[gcell] = -1;
                }
                const double uu = u0 * u0 + u1 * u1 + u2 * u2;
                for (int d = 0; d < kQ; ++d)
                    st<P>(A, (unsigned)(d * nc + z0 + c), d, (typename Prec<P>::C)feq<double>(d, rb, u0, u1, u2, uu), rho_ff);
            }
        }
        __syncthreads();
        uint2 *rtp = s.rt + M->rt_off + (long long)z * ny * nw;
        for (int w = threadIdx.x; w < ny * nw; w += blockDim.x) {
            const int j = w / nw, x0 = (w - j * nw) * 32;
            const int nb = min(32, nx - x0);
            rtp[w] = make_uint2(nb == 32 ? 0xffffffffu : ((1u << nb) - 1u), (unsigned)(j * nx + x0));
        }
        // the plane's list no longer describes the layout: the next rebuild lays it out
        if (threadIdx.x == 0) s.ccnt[pl] = -1;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// adjoint of the fluid step over frozen particle geometry
// ---------------------------------------------------------------------------
// The window's forward map is the fluid step with the node map and the particles frozen
// (positions, angular velocities; prescribed velocities V): pull streaming with
// stationary walls and the moving walls of Eq. (mem), the density faces (Sec. 2.4) with
// rho_in = rho_f + A s(t+1), and the BGK collision, all on deviations from the rest
// state as in the coupled fluid kernel.  Its discrete adjoint propagates a loss gradient
// on the probe signals backwards: lambda^n = (dS/df^n)^T lambda^{n+1} + dL/df^n.

// Pre-face populations g0 (deviation form) of fluid node (i, j, k) from the state fin,
// and the unknown directions of a density face; the moving-wall term of Eq. (mem) uses
// V_b . c_d = c_d . (V + Omega x (x - X)) of the source's particle.
template <int P>
__device__ __forceinline__ unsigned adj_gather(const AdjDev &a, const typename Prec<P>::S *fin, int i, int j, int k,
                                               int cell, typename Prec<P>::C (&g)[kQ])
{
    using C = typename Prec<P>::C;
    const MemberDev &M = a.M;
    const int nx = M.nx, ny = M.ny, nz = M.nz, nc = a.ncell;
    const int dims[3] = {nx, ny, nz};
    unsigned unk = 0u;
#pragma unroll
    for (int e = 0; e < kQ - 1; ++e) {
        int c[3] = {i - kCX[e], j - kCY[e], k - kCZ[e]};
        int kind = 0; // 0 node, 1 wall, 2 unknown
        for (int ax = 0; ax < 3; ++ax) {
            if (c[ax] < 0 || c[ax] >= dims[ax]) {
                const int f = M.bc[2 * ax + (c[ax] >= dims[ax] ? 1 : 0)];
                if (f == BC_PRESSURE) kind = 2;
                else if (f == BC_WALL) kind = max(kind, 1);
                else c[ax] = c[ax] < 0 ? c[ax] + dims[ax] : c[ax] - dims[ax];
            }
        }
        const int d = kOPP[e];
        if (kind == 2) { g[e] = C(0); unk |= 1u << e; continue; }
        if (kind == 1) { g[e] = decode_dev<P>(fin[d * nc + cell], d, a.rho_f); continue; }
        const int sc = (c[2] * ny + c[1]) * nx + c[0];
        const int q = a.own[sc];
        if (q < 0) { g[e] = decode_dev<P>(fin[e * nc + sc], e, a.rho_f); continue; }
        // (on a narrow lattice, from the link's midpoint, which fixes the image, as group_arm)
        const double h0 = M.narrow ? 0.5 * kCX[e] : 0.0, h1 = M.narrow ? 0.5 * kCY[e] : 0.0,
                     h2 = M.narrow ? 0.5 * kCZ[e] : 0.0;
        const double r0 = mimg(((double)i - h0) - a.X[3 * q], M.per[0], M.box[0]) + h0;
        const double r1 = mimg(((double)j - h1) - a.X[3 * q + 1], M.per[1], M.box[1]) + h1;
        const double r2 = mimg(((double)k - h2) - a.X[3 * q + 2], M.per[2], M.box[2]) + h2;
        const double *V = a.V + 3 * q, *W = a.W + 3 * q;
        const double u0 = V[0] + (W[1] * r2 - W[2] * r1);
        const double u1 = V[1] + (W[2] * r0 - W[0] * r2);
        const double u2 = V[2] + (W[0] * r1 - W[1] * r0);
        const double cu = (double)kCX[d] * u0 + (double)kCY[d] * u1 + (double)kCZ[d] * u2;
        g[e] = decode_dev<P>(fin[d * nc + cell], d, a.rho_f) - (C)(kMW[d] * a.rho_f) * (C)cu;
    }
    g[18] = decode_dev<P>(fin[18 * nc + cell], 18, a.rho_f);
    return unk;
}

__device__ __forceinline__ void adj_coords(const AdjDev &a, int cell, int &i, int &j, int &k)
{
    const int nxy = a.M.nx * a.M.ny;
    k = cell / nxy;
    const int rem = cell - k * nxy;
    j = rem / a.M.nx;
    i = rem - j * a.M.nx;
}

// One frozen forward step fin -> fout.
template <int P>
__global__ __launch_bounds__(256) void k_adj_step(AdjDev a, const typename Prec<P>::S *fin, typename Prec<P>::S *fout, int n)
{
    const double drho_in = a.amp * a.shape[n];
    using C = typename Prec<P>::C;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= a.ncell || a.own[cell] >= 0) return;
    int i, j, k;
    adj_coords(a, cell, i, j, k);
    C f[kQ];
    adj_gather<P>(a, fin, i, j, k, cell, f);
    if (k == 0 && a.M.bc[4] == BC_PRESSURE) zou_he<C>(f, (C)drho_in, false);
    if (k == a.M.nz - 1 && a.M.bc[5] == BC_PRESSURE) zou_he<C>(f, C(0), true);
    C drho, jx, jy, jz;
    moments<C>(f, drho, jx, jy, jz);
    const C rho = (C)a.rho_f + drho;
    const C ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const C uu = ux * ux + uy * uy + uz * uz;
    const C om = (C)a.omega;
#pragma unroll
    for (int d = 0; d < kQ; ++d) {
        const C fe = feq_dev<C>(d, drho, rho, ux, uy, uz, uu);
        store_dev<P>(fout, (unsigned)(d * a.ncell + cell), d, f[d] + om * (fe - f[d]), a.rho_f);
    }
}

// Probe signals of step n from the state f^n: one workgroup per probe plane, the plane
// average of rho - rho_f over its fluid nodes (pre-collision, after the density faces).
template <int P>
__global__ __launch_bounds__(256) void k_adj_probe(AdjDev a, const typename Prec<P>::S *fin, int n)
{
    using C = typename Prec<P>::C;
    __shared__ double red[4][8];
    const int kp = blockIdx.x;
    if (kp >= a.n_probe) return;
    const int k = a.probe_z[kp];
    const int nxy = a.M.nx * a.M.ny;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < nxy; t += blockDim.x) {
        const int cell = k * nxy + t;
        if (a.own[cell] >= 0) continue;
        const int j = t / a.M.nx, i = t - j * a.M.nx;
        C f[kQ];
        adj_gather<P>(a, fin, i, j, k, cell, f);
        if (k == 0 && a.M.bc[4] == BC_PRESSURE) zou_he<C>(f, (C)(a.amp * a.shape[n]), false);
        if (k == a.M.nz - 1 && a.M.bc[5] == BC_PRESSURE) zou_he<C>(f, C(0), true);
        C drho, jx, jy, jz;
        moments<C>(f, drho, jx, jy, jz);
        v[0] += (double)drho;
    }
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.P[(long long)n * a.n_probe + kp] = v[0] / a.probe_nfl[kp];
}

// Fluid nodes of each probe plane (one workgroup per plane).
__global__ __launch_bounds__(256) void k_adj_nfl(AdjDev a, double *nfl)
{
    __shared__ double red[4][8];
    const int kp = blockIdx.x;
    if (kp >= a.n_probe) return;
    const int nxy = a.M.nx * a.M.ny;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < nxy; t += blockDim.x)
        if (a.own[a.probe_z[kp] * nxy + t] < 0) v[0] += 1.0;
    block_sum<1>(v, red);
    if (threadIdx.x == 0) nfl[kp] = v[0];
}

// Adjoint through step n at every fluid node: from lambda^{n+1} (dL/d of the post-collision
// state) and the probe term, mu = dL/dg0 of the pre-face populations g0 of time level
// n+1.  Collision transpose: with A = sum lambda_d w_d, B = sum lambda_d w_d c_d,
// Cm = sum lambda_d w_d (c_d.u) c_d, D = sum lambda_d w_d (c_d.u)^2 (lattice units,
// 1/c_s^2 = 3), sum_d lambda_d df^eq_d/dg_e = A (1 + 1.5 u.u) - 4.5 D + (3 B + 9 Cm - 3 A u).c_e.
// The density faces are transposed by hand from their closure formulas.  Also collected:
// dL/domega = sum lambda_d (f^eq_d - g_d), dL/drho_in, and per node dL/dg0_e of every
// direction whose source is a particle (for dL/dV).
template <int P>
__global__ __launch_bounds__(256) void k_adj_mu(AdjDev a, const typename Prec<P>::S *fin,
                                                const typename Prec<P>::C *lam, typename Prec<P>::C *mu, int n)
{
    using C = typename Prec<P>::C;
    __shared__ double red[4][8];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = a.ncell;
    double acc[2] = {0.0, 0.0}; // dL/domega, dL/drho_in
    if (cell < nc && a.own[cell] < 0) {
        int i, j, k;
        adj_coords(a, cell, i, j, k);
        C g[kQ];
        const unsigned unk = adj_gather<P>(a, fin, i, j, k, cell, g);
        const int face = (k == 0 && a.M.bc[4] == BC_PRESSURE) ? 0 : ((k == a.M.nz - 1 && a.M.bc[5] == BC_PRESSURE) ? 1 : -1);
        if (face == 0) zou_he<C>(g, (C)(a.amp * a.shape[n]), false);
        if (face == 1) zou_he<C>(g, C(0), true);
        C drho, jx, jy, jz;
        moments<C>(g, drho, jx, jy, jz);
        const C rho = (C)a.rho_f + drho;
        const C ux = jx / rho, uy = jy / rho, uz = jz / rho;
        const C uu = ux * ux + uy * uy + uz * uz;
        C l[kQ];
#pragma unroll
        for (int d = 0; d < kQ; ++d) l[d] = lam[d * nc + cell];
        C A = C(0), B0 = C(0), B1 = C(0), B2 = C(0), C0 = C(0), C1 = C(0), C2 = C(0), D = C(0);
        double gw = 0.0;
#pragma unroll
        for (int d = 0; d < kQ; ++d) {
            const C wl = (C)kWd[d] * l[d];
            const C cu = (C)kCX[d] * ux + (C)kCY[d] * uy + (C)kCZ[d] * uz;
            A += wl;
            B0 += wl * (C)kCX[d]; B1 += wl * (C)kCY[d]; B2 += wl * (C)kCZ[d];
            C0 += wl * cu * (C)kCX[d]; C1 += wl * cu * (C)kCY[d]; C2 += wl * cu * (C)kCZ[d];
            D += wl * cu * cu;
            gw += (double)l[d] * (double)(feq_dev<C>(d, drho, rho, ux, uy, uz, uu) - g[d]);
        }
        acc[0] = gw;
        const C om = (C)a.omega;
        const C base = A * (C(1) + C(1.5) * uu) - C(4.5) * D;
        const C v0 = C(3) * B0 + C(9) * C0 - C(3) * A * ux;
        const C v1 = C(3) * B1 + C(9) * C1 - C(3) * A * uy;
        const C v2 = C(3) * B2 + C(9) * C2 - C(3) * A * uz;
        C pt = C(0);
        for (int kp = 0; kp < a.n_probe; ++kp)
            if (a.probe_z[kp] == k) pt += (C)(a.dLdP[(long long)n * a.n_probe + kp] / a.probe_nfl[kp]);
        C m[kQ];
#pragma unroll
        for (int e = 0; e < kQ; ++e)
            m[e] = (C(1) - om) * l[e] + om * (base + (C)kCX[e] * v0 + (C)kCY[e] * v1 + (C)kCZ[e] * v2) + pt;
        // density faces (paper index p -> m[p-1]); unknowns end with no dependence on g0
        if (face == 0) {
            const C av = m[4], bv = m[8], cv = m[12], dv = m[14], ev = m[16];
            const C R = av / C(3) + (bv + cv + dv + ev) / C(6), X = cv - bv, Y = ev - dv;
            acc[1] = (double)R * a.shape[n]; // d rho_in / dA = s(t+1)
            m[4] = m[8] = m[12] = m[14] = m[16] = C(0);
            const int s0[9] = {0, 1, 2, 3, 6, 7, 10, 11, 18}, sm[5] = {5, 9, 13, 15, 17};
#pragma unroll
            for (int q = 0; q < 9; ++q) m[s0[q]] -= R;
#pragma unroll
            for (int q = 0; q < 5; ++q) m[sm[q]] -= C(2) * R;
            m[0] += C(0.5) * X; m[6] += C(0.5) * X; m[7] += C(0.5) * X;
            m[1] -= C(0.5) * X; m[10] -= C(0.5) * X; m[11] -= C(0.5) * X;
            m[2] += C(0.5) * Y; m[6] += C(0.5) * Y; m[10] += C(0.5) * Y;
            m[3] -= C(0.5) * Y; m[7] -= C(0.5) * Y; m[11] -= C(0.5) * Y;
            m[5] += av; m[13] += bv; m[9] += cv; m[17] += dv; m[15] += ev;
        } else if (face == 1) {
            const C av = m[5], bv = m[13], cv = m[9], dv = m[17], ev = m[15];
            const C R = -av / C(3) - (bv + cv + dv + ev) / C(6), X = bv - cv, Y = dv - ev;
            m[5] = m[13] = m[9] = m[17] = m[15] = C(0);
            const int s0[9] = {0, 1, 2, 3, 6, 7, 10, 11, 18}, sp[5] = {4, 8, 12, 14, 16};
#pragma unroll
            for (int q = 0; q < 9; ++q) m[s0[q]] += R;
#pragma unroll
            for (int q = 0; q < 5; ++q) m[sp[q]] += C(2) * R;
            m[0] += C(0.5) * X; m[6] += C(0.5) * X; m[7] += C(0.5) * X;
            m[1] -= C(0.5) * X; m[10] -= C(0.5) * X; m[11] -= C(0.5) * X;
            m[2] += C(0.5) * Y; m[6] += C(0.5) * Y; m[10] += C(0.5) * Y;
            m[3] -= C(0.5) * Y; m[7] -= C(0.5) * Y; m[11] -= C(0.5) * Y;
            m[4] += av; m[8] += bv; m[12] += cv; m[14] += dv; m[16] += ev;
        }
        (void)unk;
        // moving walls: the directions whose source is a particle
        const int dims[3] = {a.M.nx, a.M.ny, a.M.nz};
#pragma unroll
        for (int e = 0; e < kQ - 1; ++e) {
            int c[3] = {i - kCX[e], j - kCY[e], k - kCZ[e]};
            bool ok = true;
            for (int ax = 0; ax < 3; ++ax)
                if (c[ax] < 0 || c[ax] >= dims[ax]) {
                    if (a.M.per[ax]) c[ax] = c[ax] < 0 ? c[ax] + dims[ax] : c[ax] - dims[ax];
                    else ok = false;
                }
            if (ok && a.own[(c[2] * dims[1] + c[1]) * dims[0] + c[0]] >= 0)
                a.macc[(long long)e * nc + cell] += (double)m[e];
        }
#pragma unroll
        for (int e = 0; e < kQ; ++e) mu[e * nc + cell] = m[e];
    }
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
        a.acc_w[blockIdx.x] += acc[0];
        a.acc_a[blockIdx.x] += acc[1];
    }
}

// lambda^n from mu: every post-collision population f~_e(y) has one consumer, the node
// y + c_e pulling direction e, or y itself bouncing it back from a wall or a particle;
// populations leaving through a density face have none.
template <int P>
__global__ __launch_bounds__(256) void k_adj_pull(AdjDev a, const typename Prec<P>::C *mu, typename Prec<P>::C *lam)
{
    using C = typename Prec<P>::C;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = a.ncell;
    if (cell >= nc) return;
    if (a.own[cell] >= 0) {
#pragma unroll
        for (int e = 0; e < kQ; ++e) lam[e * nc + cell] = C(0);
        return;
    }
    int i, j, k;
    adj_coords(a, cell, i, j, k);
    const int dims[3] = {a.M.nx, a.M.ny, a.M.nz};
#pragma unroll
    for (int e = 0; e < kQ - 1; ++e) {
        int c[3] = {i + kCX[e], j + kCY[e], k + kCZ[e]};
        int kind = 0;
        for (int ax = 0; ax < 3; ++ax) {
            if (c[ax] < 0 || c[ax] >= dims[ax]) {
                const int f = a.M.bc[2 * ax + (c[ax] >= dims[ax] ? 1 : 0)];
                if (f == BC_PRESSURE) kind = 2;
                else if (f == BC_WALL) kind = max(kind, 1);
                else c[ax] = c[ax] < 0 ? c[ax] + dims[ax] : c[ax] - dims[ax];
            }
        }
        C v = C(0);
        if (kind == 1) v = mu[kOPP[e] * nc + cell];
        else if (kind == 0) {
            const int x = (c[2] * dims[1] + c[1]) * dims[0] + c[0];
            v = (a.own[x] >= 0) ? mu[kOPP[e] * nc + cell] : mu[e * nc + x];
        }
        lam[e * nc + cell] = v;
    }
    lam[18 * nc + cell] = mu[18 * nc + cell];
}

// dL/dV_q = sum over q's links (x, e) of -2 (w_d / c_s^2) rho_f c_d dL/dg0_e(x), d = e*:
// one workgroup per particle over the nodes within R_q + 2 of X_q, in a fixed order.
__global__ __launch_bounds__(256) void k_adj_vgrad(AdjDev a)
{
    __shared__ double red[4][8];
    const int q = blockIdx.x;
    if (q >= a.np) return;
    const MemberDev &M = a.M;
    const int dims[3] = {M.nx, M.ny, M.nz};
    int lo[3], ext[3];
    for (int ax = 0; ax < 3; ++ax) axis_range(a.X[3 * q + ax], a.R[q] + 2.0, dims[ax], M.per[ax], lo[ax], ext[ax]);
    const int tot = ext[0] * ext[1] * ext[2];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int ii = wrapc(lo[0] + idx % ext[0], dims[0]);
        const int jj = wrapc(lo[1] + (idx / ext[0]) % ext[1], dims[1]);
        const int kk = wrapc(lo[2] + idx / (ext[0] * ext[1]), dims[2]);
        const int x = (kk * dims[1] + jj) * dims[0] + ii;
        if (a.own[x] >= 0) continue;
        for (int e = 0; e < kQ - 1; ++e) {
            int c[3] = {ii - kCXd[e], jj - kCYd[e], kk - kCZd[e]};
            bool ok = true;
            for (int ax = 0; ax < 3; ++ax)
                if (c[ax] < 0 || c[ax] >= dims[ax]) {
                    if (M.per[ax]) c[ax] = c[ax] < 0 ? c[ax] + dims[ax] : c[ax] - dims[ax];
                    else ok = false;
                }
            if (!ok || a.own[(c[2] * dims[1] + c[1]) * dims[0] + c[0]] != q) continue;
            // d g0_e / dV = -2 (w_d / c_s^2) rho_f c_d with c_d = -c_e and w_d = w_e
            const int c2 = kCXd[e] * kCXd[e] + kCYd[e] * kCYd[e] + kCZd[e] * kCZd[e];
            const double w = (c2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
            const double f = 2.0 * w / kCS2 * a.rho_f * a.macc[(long long)e * a.ncell + x];
            acc[0] += f * kCXd[e];
            acc[1] += f * kCYd[e];
            acc[2] += f * kCZd[e];
        }
    }
    block_sum<3>(acc, red);
    if (threadIdx.x == 0)
        for (int ax = 0; ax < 3; ++ax) a.gv[3 * q + ax] = acc[ax];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <bool CMP, bool NR>
void *fluid_ptr(int prec)
{
    switch (prec) {
    case PREC_FP64: return (void *)&k_fluid<PREC_FP64, CMP, NR>;
    case PREC_FP32: return (void *)&k_fluid<PREC_FP32, CMP, NR>;
    case PREC_FP16DEV: return (void *)&k_fluid<PREC_FP16DEV, CMP, NR>;
    default: return (void *)&k_fluid<PREC_BF16DEV, CMP, NR>;
    }
}
void *fluid_kernel_ptr(int prec, int compact, int narrow)
{
    if (narrow) return compact ? fluid_ptr<true, true>(prec) : fluid_ptr<false, true>(prec);
    return compact ? fluid_ptr<true, false>(prec) : fluid_ptr<false, false>(prec);
}
template <bool NR>
void *links_ptr(int prec)
{
    switch (prec) {
    case PREC_FP64: return (void *)&k_links<PREC_FP64, NR>;
    case PREC_FP32: return (void *)&k_links<PREC_FP32, NR>;
    case PREC_FP16DEV: return (void *)&k_links<PREC_FP16DEV, NR>;
    default: return (void *)&k_links<PREC_BF16DEV, NR>;
    }
}
void *links_kernel_ptr(int prec, int narrow) { return narrow ? links_ptr<true>(prec) : links_ptr<false>(prec); }
void *motion_kernel_ptr() { return (void *)&k_motion; }
void *remap_kernel_ptr_prec(int prec)
{
    switch (prec) {
    case PREC_FP64: return (void *)&k_remap<PREC_FP64>;
    case PREC_FP32: return (void *)&k_remap<PREC_FP32>;
    case PREC_FP16DEV: return (void *)&k_remap<PREC_FP16DEV>;
    default: return (void *)&k_remap<PREC_BF16DEV>;
    }
}
int links_grid(const DevSet &s) { return max(s.ptot * kChunks, 1); }
int refresh_grid(const DevSet &) { return kRefreshBlocks; }
void *refresh_kernel_ptr(int prec)
{
    switch (prec) {
    case PREC_FP64: return reinterpret_cast<void *>(&k_refresh<PREC_FP64>);
    case PREC_FP32: return reinterpret_cast<void *>(&k_refresh<PREC_FP32>);
    case PREC_FP16DEV: return reinterpret_cast<void *>(&k_refresh<PREC_FP16DEV>);
    default: return reinterpret_cast<void *>(&k_refresh<PREC_BF16DEV>);
    }
}

hipError_t launch_refresh(int prec, const DevSet &s, hipStream_t st)
{
    const dim3 g(refresh_grid(s)), b(256);
    switch (prec) {
    case PREC_FP64: hipLaunchKernelGGL(k_refresh<PREC_FP64>, g, b, 0, st, s); break;
    case PREC_FP32: hipLaunchKernelGGL(k_refresh<PREC_FP32>, g, b, 0, st, s); break;
    case PREC_FP16DEV: hipLaunchKernelGGL(k_refresh<PREC_FP16DEV>, g, b, 0, st, s); break;
    default: hipLaunchKernelGGL(k_refresh<PREC_BF16DEV>, g, b, 0, st, s); break;
    }
    return hipGetLastError();
}
int motion_grid(const DevSet &s) { return max((s.ptot + kMotionWaves - 1) / kMotionWaves, 1); }
int remap_grid(const DevSet &s) { return max((s.ptot + kRemapWaves - 1) / kRemapWaves + s.nprobe_total, 1); }

template <bool CMP, bool NR>
void *records_ptr(int prec)
{
    switch (prec) {
    case PREC_FP64: return (void *)&k_records<PREC_FP64, CMP, NR>;
    case PREC_FP32: return (void *)&k_records<PREC_FP32, CMP, NR>;
    case PREC_FP16DEV: return (void *)&k_records<PREC_FP16DEV, CMP, NR>;
    default: return (void *)&k_records<PREC_BF16DEV, CMP, NR>;
    }
}
void *records_kernel_ptr(int prec, int compact, int narrow)
{
    if (narrow) return compact ? records_ptr<true, true>(prec) : records_ptr<false, true>(prec);
    return compact ? records_ptr<true, false>(prec) : records_ptr<false, false>(prec);
}
int records_grid(const DevSet &s) { return rebuild_blocks(s) + s.tiles_total; }
hipError_t launch_records(int prec, const DevSet &s, hipStream_t st)
{
    hipLaunchKernelGGL(reinterpret_cast<void (*)(DevSet)>(records_kernel_ptr(prec, s.compact, s.narrow)),
                       dim3(records_grid(s)), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_fluid(int prec, const DevSet &s, hipStream_t st)
{
    hipLaunchKernelGGL(reinterpret_cast<void (*)(DevSet)>(fluid_kernel_ptr(prec, s.compact, s.narrow)),
                       dim3(s.tiles_total), dim3(256), 0, st, s);
    return hipGetLastError();
}

int links_block() { return kLinksBlock; }

hipError_t launch_links(int prec, const DevSet &s, hipStream_t st)
{
    const int mode = 0, only = -1;
    hipLaunchKernelGGL(reinterpret_cast<void (*)(DevSet, int, int)>(links_kernel_ptr(prec, s.narrow)),
                       dim3(links_grid(s)), dim3(kLinksBlock), 0, st, s, mode, only);
    return hipGetLastError();
}

hipError_t launch_motion(const DevSet &s, int mode, int only_member, hipStream_t st)
{
    hipLaunchKernelGGL(k_motion, dim3(motion_grid(s)), dim3(256), 0, st, s, mode, only_member);
    return hipGetLastError();
}

hipError_t launch_remap_prec(int prec, const DevSet &s, int mode, int only_member, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64: hipLaunchKernelGGL(k_remap<PREC_FP64>, dim3(remap_grid(s)), dim3(256), 0, st, s, mode, only_member); break;
    case PREC_FP32: hipLaunchKernelGGL(k_remap<PREC_FP32>, dim3(remap_grid(s)), dim3(256), 0, st, s, mode, only_member); break;
    case PREC_FP16DEV: hipLaunchKernelGGL(k_remap<PREC_FP16DEV>, dim3(remap_grid(s)), dim3(256), 0, st, s, mode, only_member); break;
    default: hipLaunchKernelGGL(k_remap<PREC_BF16DEV>, dim3(remap_grid(s)), dim3(256), 0, st, s, mode, only_member); break;
    }
    return hipGetLastError();
}

int adj_blocks(const AdjDev &a) { return (a.ncell + 255) / 256; }

template <int P> using StoreT = typename Prec<P>::S;
template <int P> using CompT = typename Prec<P>::C;

hipError_t launch_adj_step(int prec, const AdjDev &a, const void *fin, void *fout, int n, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64:
        hipLaunchKernelGGL(k_adj_step<PREC_FP64>, dim3(adj_blocks(a)), dim3(256), 0, st, a,
                           (const StoreT<PREC_FP64> *)fin, (StoreT<PREC_FP64> *)fout, n);
        break;
    case PREC_FP32:
        hipLaunchKernelGGL(k_adj_step<PREC_FP32>, dim3(adj_blocks(a)), dim3(256), 0, st, a,
                           (const StoreT<PREC_FP32> *)fin, (StoreT<PREC_FP32> *)fout, n);
        break;
    case PREC_FP16DEV:
        hipLaunchKernelGGL(k_adj_step<PREC_FP16DEV>, dim3(adj_blocks(a)), dim3(256), 0, st, a,
                           (const StoreT<PREC_FP16DEV> *)fin, (StoreT<PREC_FP16DEV> *)fout, n);
        break;
    default:
        hipLaunchKernelGGL(k_adj_step<PREC_BF16DEV>, dim3(adj_blocks(a)), dim3(256), 0, st, a,
                           (const StoreT<PREC_BF16DEV> *)fin, (StoreT<PREC_BF16DEV> *)fout, n);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_adj_probe(int prec, const AdjDev &a, const void *fin, int n, hipStream_t st)
{
    const int g = a.n_probe > 0 ? a.n_probe : 1;
    switch (prec) {
    case PREC_FP64: hipLaunchKernelGGL(k_adj_probe<PREC_FP64>, dim3(g), dim3(256), 0, st, a, (const StoreT<PREC_FP64> *)fin, n); break;
    case PREC_FP32: hipLaunchKernelGGL(k_adj_probe<PREC_FP32>, dim3(g), dim3(256), 0, st, a, (const StoreT<PREC_FP32> *)fin, n); break;
    case PREC_FP16DEV: hipLaunchKernelGGL(k_adj_probe<PREC_FP16DEV>, dim3(g), dim3(256), 0, st, a, (const StoreT<PREC_FP16DEV> *)fin, n); break;
    default: hipLaunchKernelGGL(k_adj_probe<PREC_BF16DEV>, dim3(g), dim3(256), 0, st, a, (const StoreT<PREC_BF16DEV> *)fin, n); break;
    }
    return hipGetLastError();
}

hipError_t launch_adj_mu(int prec, const AdjDev &a, const void *fin, const void *lam, void *mu, int n, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64:
        hipLaunchKernelGGL(k_adj_mu<PREC_FP64>, dim3(adj_blocks(a)), dim3(256), 0, st, a, (const StoreT<PREC_FP64> *)fin,
                           (const CompT<PREC_FP64> *)lam, (CompT<PREC_FP64> *)mu, n);
        break;
    case PREC_FP32:
        hipLaunchKernelGGL(k_adj_mu<PREC_FP32>, dim3(adj_blocks(a)), dim3(256), 0, st, a, (const StoreT<PREC_FP32> *)fin,
                           (const CompT<PREC_FP32> *)lam, (CompT<PREC_FP32> *)mu, n);
        break;
    case PREC_FP16DEV:
        hipLaunchKernelGGL(k_adj_mu<PREC_FP16DEV>, dim3(adj_blocks(a)), dim3(256), 0, st, a, (const StoreT<PREC_FP16DEV> *)fin,
                           (const CompT<PREC_FP16DEV> *)lam, (CompT<PREC_FP16DEV> *)mu, n);
        break;
    default:
        hipLaunchKernelGGL(k_adj_mu<PREC_BF16DEV>, dim3(adj_blocks(a)), dim3(256), 0, st, a, (const StoreT<PREC_BF16DEV> *)fin,
                           (const CompT<PREC_BF16DEV> *)lam, (CompT<PREC_BF16DEV> *)mu, n);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_adj_pull(int prec, const AdjDev &a, const void *mu, void *lam, hipStream_t st)
{
    if (prec == PREC_FP64)
        hipLaunchKernelGGL(k_adj_pull<PREC_FP64>, dim3(adj_blocks(a)), dim3(256), 0, st, a, (const double *)mu, (double *)lam);
    else
        hipLaunchKernelGGL(k_adj_pull<PREC_FP32>, dim3(adj_blocks(a)), dim3(256), 0, st, a, (const float *)mu, (float *)lam);
    return hipGetLastError();
}

hipError_t launch_adj_vgrad(const AdjDev &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_vgrad, dim3(a.np > 0 ? a.np : 1), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_nfl(const AdjDev &a, double *nfl, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_nfl, dim3(a.n_probe > 0 ? a.n_probe : 1), dim3(256), 0, st, a, nfl);
    return hipGetLastError();
}

hipError_t launch_init_pops(int prec, const DevSet &s, long long total_cells, hipStream_t st)
{
    const unsigned grid = (unsigned)((total_cells + 255) / 256);
    if (grid == 0) return hipSuccess;
    switch (prec) {
    case PREC_FP64: hipLaunchKernelGGL(k_init_pops<PREC_FP64>, dim3(grid), dim3(256), 0, st, s, total_cells); break;
    case PREC_FP32: hipLaunchKernelGGL(k_init_pops<PREC_FP32>, dim3(grid), dim3(256), 0, st, s, total_cells); break;
    case PREC_FP16DEV: hipLaunchKernelGGL(k_init_pops<PREC_FP16DEV>, dim3(grid), dim3(256), 0, st, s, total_cells); break;
    default: hipLaunchKernelGGL(k_init_pops<PREC_BF16DEV>, dim3(grid), dim3(256), 0, st, s, total_cells); break;
    }
    return hipGetLastError();
}

hipError_t launch_fields(int prec, const DevSet &s, int m, long long ncell, double *out, hipStream_t st)
{
    const dim3 g((unsigned)((ncell + 255) / 256)), b(256);
    switch (prec) {
    case PREC_FP64: hipLaunchKernelGGL(k_fields<PREC_FP64>, g, b, 0, st, s, m, out); break;
    case PREC_FP32: hipLaunchKernelGGL(k_fields<PREC_FP32>, g, b, 0, st, s, m, out); break;
    case PREC_FP16DEV: hipLaunchKernelGGL(k_fields<PREC_FP16DEV>, g, b, 0, st, s, m, out); break;
    default: hipLaunchKernelGGL(k_fields<PREC_BF16DEV>, g, b, 0, st, s, m, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_expand(int prec, const DevSet &s, hipStream_t st)
{
    const dim3 g(max(s.nplanes, 1));
    switch (prec) {
    case PREC_FP64: hipLaunchKernelGGL(k_expand<PREC_FP64>, g, dim3(256), 0, st, s); break;
    case PREC_FP32: hipLaunchKernelGGL(k_expand<PREC_FP32>, g, dim3(256), 0, st, s); break;
    case PREC_FP16DEV: hipLaunchKernelGGL(k_expand<PREC_FP16DEV>, g, dim3(256), 0, st, s); break;
    default: hipLaunchKernelGGL(k_expand<PREC_BF16DEV>, g, dim3(256), 0, st, s); break;
    }
    return hipGetLastError();
}

} // namespace lbdem
