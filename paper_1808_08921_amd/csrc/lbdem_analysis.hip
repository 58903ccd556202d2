// lbdem_analysis.hip -- dispersion analysis of probe records (Sec. 3.2).
//
// Space-time DFT of a probe record x[t][z] on a chosen (omega, kappa) grid, the ridge of its
// spectrum, and the fit of the stationary lossy wave of Eq. (1Dwave).  FP64 throughout.
//
// Time stage: one lane per kMPL frequencies omega_m and one wave per group of kZB columns; the
// lanes of a wave share each record row (staged in LDS, read as broadcasts) and advance
// their phase factor exp(-j omega_m t) by a complex rotation, re-anchored with an exact
// sincos every kAnchor steps, so the time stage costs about two FMAs per sample and
// frequency.  Time is split into chunks whose partial sums are added in chunk order
// (deterministic), then the space stage multiplies by a table of exp(j kappa_n z).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>
#include <stdint.h>

#include "lbdem_internal.hpp"

namespace lbdem {

namespace {

constexpr int kZB = 8;        // columns per wave in the time stage
constexpr int kAnchor = 64;   // steps between exact phase anchors (one record row per lane)
constexpr int kMPL = 2;       // frequencies per lane in the time stage
constexpr int kTargetBlocks = 1024;

__device__ inline double2 cmul_acc(double2 acc, double2 a, double2 b)
{
    // acc + a * b (complex)
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
    return acc;
}

__global__ __launch_bounds__(256) void k_dft_time(const double *__restrict__ x, long long nt, int nz, double t0,
                                                  double w0, double dw, int nw, int nwb, long long chunk,
                                                  double2 *__restrict__ part)
{
    // per wave: kAnchor record rows x kZB columns, written by the lanes and read back as
    // broadcasts; the next rows are loaded into registers while the current ones are used
    __shared__ double2 tile[4][kAnchor * kZB / 2];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int mb = blockIdx.x % nwb;
    const long long c = blockIdx.x / nwb;
    const int m0 = mb * 64 * kMPL + lane;  // the lane's frequencies m0 + 64 f
    const int z0 = (blockIdx.y * (blockDim.x >> 6) + wv) * kZB;
    if (z0 >= nz) return;  // whole wave; the kernel has no block-wide barrier
    const int zn = min(kZB, nz - z0);
    const long long ta = c * chunk;
    const long long tb = min(ta + chunk, nt);
    double om[kMPL], rs[kMPL], rc[kMPL];
#pragma unroll
    for (int f = 0; f < kMPL; ++f) {
        om[f] = w0 + (double)(m0 + 64 * f) * dw;
        sincos(om[f], &rs[f], &rc[f]);
    }
    double ar[kMPL][kZB], ai[kMPL][kZB];
#pragma unroll
    for (int f = 0; f < kMPL; ++f)
#pragma unroll
        for (int q = 0; q < kZB; ++q) ar[f][q] = ai[f][q] = 0.0;
    // lane -> row `lane` of a tile, all kZB columns
    double v[kZB];
    auto fetch = [&](long long t) {
        const long long u = t + lane;
#pragma unroll
        for (int q = 0; q < kZB; ++q) v[q] = (u < tb && q < zn) ? x[u * nz + z0 + q] : 0.0;
    };
    double2 *tw = tile[wv];
    fetch(ta);
    for (long long t = ta; t < tb; t += kAnchor) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int h = 0; h < kZB / 2; ++h) tw[lane * (kZB / 2) + h] = make_double2(v[2 * h], v[2 * h + 1]);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (t + kAnchor < tb) fetch(t + kAnchor);
        double s[kMPL], co[kMPL];
#pragma unroll
        for (int f = 0; f < kMPL; ++f) sincos(om[f] * (t0 + (double)t), &s[f], &co[f]);  // exp(-j theta) = co - j s
        const int nr = (int)min((long long)kAnchor, tb - t);
        for (int r = 0; r < nr; ++r) {
#pragma unroll
            for (int h = 0; h < kZB / 2; ++h) {
                const double2 v = tw[r * (kZB / 2) + h];
#pragma unroll
                for (int f = 0; f < kMPL; ++f) {
                    ar[f][2 * h] = fma(v.x, co[f], ar[f][2 * h]);
                    ai[f][2 * h] = fma(-v.x, s[f], ai[f][2 * h]);
                    ar[f][2 * h + 1] = fma(v.y, co[f], ar[f][2 * h + 1]);
                    ai[f][2 * h + 1] = fma(-v.y, s[f], ai[f][2 * h + 1]);
                }
            }
            // exp(-j (theta + omega)) = (co - j s)(rc - j rs)
#pragma unroll
            for (int f = 0; f < kMPL; ++f) {
                const double cn = fma(co[f], rc[f], -s[f] * rs[f]);
                const double sn = fma(s[f], rc[f], co[f] * rs[f]);
                co[f] = cn;
                s[f] = sn;
            }
        }
    }
#pragma unroll
    for (int f = 0; f < kMPL; ++f) {
        const int m = m0 + 64 * f;
        if (m < nw) {
            double2 *dst = part + ((size_t)c * nw + m) * nz + z0;
#pragma unroll
            for (int q = 0; q < kZB; ++q)
                if (q < zn) dst[q] = make_double2(ar[f][q], ai[f][q]);
        }
    }
}

// G[m][z] = sum over chunks, in chunk order
__global__ __launch_bounds__(256) void k_dft_sum(const double2 *__restrict__ part, long long nmz, int nchunk,
                                                 double2 *__restrict__ G)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nmz) return;
    double2 a = part[i];
#pragma unroll 8
    for (int c = 1; c < nchunk; ++c) {
        const double2 b = part[(size_t)c * nmz + i];
        a.x += b.x;
        a.y += b.y;
    }
    G[i] = a;
}

// E[z][n] = exp(j kappa_n zpos[z])
__global__ __launch_bounds__(256) void k_phase(const double *__restrict__ zpos, int nz, double k0, double dk, int nk,
                                               double2 *__restrict__ E)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)nz * nk) return;
    const int z = (int)(i / nk), n = (int)(i % nk);
    const double ka = k0 + (double)n * dk;
    double s, c;
    sincos(ka * zpos[z], &s, &c);
    E[i] = make_double2(c, s);
}

// F[m][n] = sum_z G[m][z] E[z][n]
__global__ __launch_bounds__(256) void k_dft_space(const double2 *__restrict__ G, const double2 *__restrict__ E,
                                                   int nz, int nk, int nkb, double2 *__restrict__ F)
{
    const int m = blockIdx.x / nkb;
    const int n = (blockIdx.x % nkb) * 256 + threadIdx.x;
    if (n >= nk) return;
    const double2 *g = G + (size_t)m * nz;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
    for (int z = 0; z < nz; ++z) acc = cmul_acc(acc, g[z], E[(size_t)z * nk + n]);
    F[(size_t)m * nk + n] = acc;
}

// ridge[m] = first n of the largest re^2 + im^2 in row m; one wave per row
__global__ __launch_bounds__(64) void k_ridge(const double2 *__restrict__ F, int nk, int *__restrict__ ridge)
{
    const int m = blockIdx.x;
    const int lane = threadIdx.x;
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int n = lane; n < nk; n += 64) {
        const double2 f = F[(size_t)m * nk + n];
        const double p = f.x * f.x + f.y * f.y;
        if (p > best) {
            best = p;
            bi = n;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    if (lane == 0) ridge[m] = bi == 0x7fffffff ? -1 : bi;
}

// partial sums of x[t][z] exp(-j omega (t0 + t)) over the steps of slice s: one wave per
// (slice, column), lanes over the steps, a fixed-order butterfly across the lanes
__global__ __launch_bounds__(64) void k_harmonic(const double *__restrict__ x, long long nt, int nz, double t0,
                                                 double omega, long long chunk, double2 *__restrict__ ph)
{
    const int z = blockIdx.x, s_ = blockIdx.y;
    const long long ta = (long long)s_ * chunk;
    const long long tb = min(ta + chunk, nt);
    double ar = 0.0, ai = 0.0;
    for (long long t = ta + threadIdx.x; t < tb; t += 64) {
        double s, c;
        sincos(omega * (t0 + (double)t), &s, &c);
        const double v = x[t * nz + z];
        ar = fma(v, c, ar);
        ai = fma(-v, s, ai);
    }
    for (int off = 32; off > 0; off >>= 1) {
        ar += __shfl_xor(ar, off);
        ai += __shfl_xor(ai, off);
    }
    if (threadIdx.x == 0) ph[(size_t)z * gridDim.y + s_] = make_double2(ar, ai);
}

// P[z] = (2 / nt) (sum of the slices in order); log |P| and arg P per column in parallel,
// then one lane unwraps the phases along the columns and fits the two straight lines
constexpr int kFitLds = 2048;

__global__ __launch_bounds__(1024) void k_wave_fit(const double2 *__restrict__ ph, int nslice, long long nt,
                                                  const double *zpos, int nz, double omega, double2 *la,
                                                  double *__restrict__ out)
{
    const double sc = 2.0 / (double)nt;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    for (int z = wv; z < nz; z += nwv) {
        // one wave per column: lanes over the slices, then a fixed-order butterfly
        double pr = 0.0, pi_ = 0.0;
        for (int q = lane; q < nslice; q += 64) {
            const double2 v = ph[(size_t)z * nslice + q];
            pr += v.x;
            pi_ += v.y;
        }
        for (int off = 32; off > 0; off >>= 1) {
            pr += __shfl_xor(pr, off);
            pi_ += __shfl_xor(pi_, off);
        }
        pr *= sc;
        pi_ *= sc;
        // log |P| is -inf for P = 0: such a column carries no phase and is left out
        if (lane == 0) la[z] = make_double2(log(hypot(pr, pi_)), atan2(pi_, pr));
    }
    // the serial part reads LDS copies of (log |P|, arg P) and zpos when they fit
    __shared__ double2 s_la[kFitLds];
    __shared__ double s_z[kFitLds];
    __syncthreads();
    const bool use_lds = nz <= kFitLds;
    if (use_lds) {
        for (int z = threadIdx.x; z < nz; z += blockDim.x) {
            s_la[z] = la[z];
            s_z[z] = zpos[z];
        }
        __syncthreads();
        la = s_la;
        zpos = s_z;
    }
    if (threadIdx.x != 0) return;
    const double pi = 3.14159265358979323846;
    const double ninf = -__builtin_inf();
    double sz = 0.0, sm = 0.0, sp = 0.0;
    int cnt = 0;
    {
        double prev = 0.0, run = 0.0;
        for (int z = 0; z < nz; ++z) {
            const double2 v = la[z];
            if (v.x == ninf) continue;
            if (cnt == 0) {
                run = v.y;
            } else {
                double d = v.y - prev;
                if (d > pi) d -= 2.0 * pi;
                else if (d < -pi) d += 2.0 * pi;
                run += d;
            }
            prev = v.y;
            sz += zpos[z];
            sm += v.x;
            sp += run;
            ++cnt;
        }
    }
    if (cnt < 2) {
        const double nan = __builtin_nan("");
        for (int i = 0; i < 5; ++i) out[i] = nan;
        out[5] = (double)cnt;
        return;
    }
    const double zb = sz / cnt, mb = sm / cnt, pb = sp / cnt;
    double szz = 0.0, szm = 0.0, szp = 0.0;
    {
        double prev = 0.0, run = 0.0;
        int k = 0;
        for (int z = 0; z < nz; ++z) {
            const double2 v = la[z];
            if (v.x == ninf) continue;
            if (k == 0) {
                run = v.y;
            } else {
                double d = v.y - prev;
                if (d > pi) d -= 2.0 * pi;
                else if (d < -pi) d += 2.0 * pi;
                run += d;
            }
            prev = v.y;
            ++k;
            const double dz = zpos[z] - zb;
            szz += dz * dz;
            szm += dz * (v.x - mb);
            szp += dz * (run - pb);
        }
    }
    const double s_mag = szm / szz, s_ph = szp / szz;
    const double i_mag = mb - s_mag * zb, i_ph = pb - s_ph * zb;
    const double amp = exp(i_mag);
    out[0] = amp * cos(i_ph);
    out[1] = amp * sin(i_ph);
    out[2] = -s_mag;
    out[3] = -s_ph;
    out[4] = omega / (-s_ph);
    out[5] = (double)cnt;
}

// x[i][p] = mean rho' (quantity 0) or sum rho u_z / sum rho (quantity 1) of probe plane p at
// step first + i, from the probe ring records (count, sum rho', sum rho u_z, sum rho)
__global__ __launch_bounds__(256) void k_probe_signal(const double *__restrict__ ring, int ring_len, int nprobe,
                                                      long long first, long long n, int quantity,
                                                      double *__restrict__ x)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nprobe) return;
    const long long s = i / nprobe;
    const int p = (int)(i % nprobe);
    const long long slot = (first + s) % ring_len;
    const double *rec = ring + (slot * nprobe + p) * 4;
    const double cnt = rec[0];
    x[i] = cnt > 0.0 ? (quantity == 0 ? rec[1] / cnt : rec[2] / rec[3]) : 0.0;
}

// x[i][l] = average of velocity component `component` over the particles of layer l after
// step first + i, from the particle-velocity ring; the members of layer l are
// members[start[l] .. start[l + 1]) in index order (a fixed summation order)
__global__ __launch_bounds__(256) void k_particle_signal(const double *__restrict__ ring, int ring_len, int ptot,
                                                         int p_off, long long first, long long n,
                                                         const int *__restrict__ start,
                                                         const int *__restrict__ members, int n_layers,
                                                         int component, double *__restrict__ x)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n_layers) return;
    const long long st = i / n_layers;
    const int l = (int)(i - st * n_layers);
    const double *rec = ring + ((first + st) % ring_len) * (long long)ptot * 3;
    const int a = start[l], b = start[l + 1];
    double sum = 0.0;
    for (int k = a; k < b; ++k) sum += rec[(long long)(p_off + members[k]) * 3 + component];
    x[i] = b > a ? sum / (double)(b - a) : 0.0;
}

inline long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

}  // namespace

DftPlan dft_plan(long long nt, int nz, int nw, int nk)
{
    DftPlan p;
    p.nwb = (int)ceil_div(nw, 64 * kMPL);
    const int wpb = (int)std::min<long long>(4, ceil_div(nz, kZB));  // waves per block
    p.threads = 64 * wpb;
    p.nzb = (int)ceil_div(nz, (long long)wpb * kZB);
    long long nchunk = std::max<long long>(1, kTargetBlocks / ((long long)p.nwb * p.nzb));
    nchunk = std::min(nchunk, std::max<long long>(1, ceil_div(nt, kAnchor)));
    long long chunk = ceil_div(nt, nchunk);
    chunk = ceil_div(chunk, kAnchor) * kAnchor;
    p.chunk = chunk;
    p.nchunk = (int)ceil_div(nt, chunk);
    const size_t sz2 = sizeof(double2);
    p.part_bytes = ((size_t)p.nchunk * nw * nz * sz2 + 255) / 256 * 256;
    p.g_bytes = ((size_t)nw * nz * sz2 + 255) / 256 * 256;
    p.e_bytes = ((size_t)nz * nk * sz2 + 255) / 256 * 256;
    return p;
}

hipError_t launch_st_dft(const DftPlan &p, const double *x, long long nt, int nz, const double *zpos, double t0,
                         double w0, double dw, int nw, double k0, double dk, int nk, double *F, int *ridge,
                         void *work, hipStream_t st)
{
    char *w = (char *)work;
    double2 *part = (double2 *)w;
    double2 *G = (double2 *)(w + p.part_bytes);
    double2 *E = (double2 *)(w + p.part_bytes + p.g_bytes);
    hipLaunchKernelGGL(k_dft_time, dim3((unsigned)((long long)p.nwb * p.nchunk), p.nzb), dim3(p.threads), 0, st, x,
                       nt, nz, t0, w0, dw, nw, p.nwb, p.chunk, part);
    const long long nmz = (long long)nw * nz;
    hipLaunchKernelGGL(k_dft_sum, dim3((unsigned)ceil_div(nmz, 256)), dim3(256), 0, st, (const double2 *)part, nmz,
                       p.nchunk, G);
    hipLaunchKernelGGL(k_phase, dim3((unsigned)ceil_div((long long)nz * nk, 256)), dim3(256), 0, st, zpos, nz, k0, dk,
                       nk, E);
    const int nkb = (int)ceil_div(nk, 256);
    hipLaunchKernelGGL(k_dft_space, dim3((unsigned)((long long)nw * nkb)), dim3(256), 0, st, (const double2 *)G,
                       (const double2 *)E, nz, nk, nkb, (double2 *)F);
    if (ridge) hipLaunchKernelGGL(k_ridge, dim3(nw), dim3(64), 0, st, (const double2 *)F, nk, ridge);
    return hipGetLastError();
}

hipError_t launch_wave_fit(const double *x, long long nt, int nz, const double *zpos, double t0, double omega,
                           double *out, void *work, hipStream_t st)
{
    // the slices of the time stage's plan for one frequency: their partial sums fill the
    // plan's partials region, the per-column (log |P|, arg P) its time-stage sums region
    const DftPlan p = dft_plan(nt, nz, 1, 1);
    double2 *ph = (double2 *)work;
    double2 *la = (double2 *)((char *)work + p.part_bytes);
    hipLaunchKernelGGL(k_harmonic, dim3(nz, p.nchunk), dim3(64), 0, st, x, nt, nz, t0, omega, p.chunk, ph);
    hipLaunchKernelGGL(k_wave_fit, dim3(1), dim3(1024), 0, st, (const double2 *)ph, p.nchunk, nt, zpos, nz, omega, la,
                       out);
    return hipGetLastError();
}

hipError_t launch_particle_signal(const double *ring, int ring_len, int ptot, int p_off, long long first,
                                  long long n, const int *start, const int *members, int n_layers, int component,
                                  double *x, hipStream_t st)
{
    const long long tot = n * n_layers;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_particle_signal, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, st, ring, ring_len, ptot,
                       p_off, first, n, start, members, n_layers, component, x);
    return hipGetLastError();
}

hipError_t launch_probe_signal(const double *ring, int ring_len, int nprobe, long long first, long long n,
                               int quantity, double *x, hipStream_t st)
{
    const long long tot = n * nprobe;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_signal, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, st, ring, ring_len, nprobe,
                       first, n, quantity, x);
    return hipGetLastError();
}

// Scratch of the allocation-free fit (lbdem_wave_fit_noalloc): a file-scope device array,
// one copy per GPU held until the process ends.  Host code never uses the array's name as
// an address: its device address is taken once per device with hipGetSymbolAddress (with
// that device current) and kept.  Calls on one GPU share the array, so calls that overlap
// on one GPU race; the fit's kernels write every scratch value before reading it.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace lbdem
