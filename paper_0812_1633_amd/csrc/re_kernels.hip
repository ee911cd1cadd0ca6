// re_kernels.hip -- lockstep kernels of the replica-exchange LJ engine:
// one launch per phase for a batch of replicas (the batched lockstep form)
// or for one replica (the plain per-replica form), plus the exchange kernel
// and the test hooks.  The per-atom arithmetic lives in re_device.hpp.
#include "re_device.hpp"

namespace re {

template <class P>
__global__ __launch_bounds__(256) void k_start(DevState d, StepArgs sa)
{
    const int b = sa.blk_off + blockIdx.x;
    const int r = sa.tab.rep[b];
    if (r < 0) return;
    const RepDev rd = d.rep[r];
    const int i = sa.tab.a0[b] + threadIdx.x;
    if (i >= rd.N) return;
    start_atom<P>(d, sa, rd, r, i, sa.cur, sa.step, sa.apply_alpha != 0);
}

// One workgroup per replica; runs only where the update flag of this parity
// is set (or everywhere with force_all).
template <class P>
__global__ __launch_bounds__(kReorderThreads) void k_reorder(DevState d, StepArgs sa)
{
    const int r = sa.r0 + blockIdx.x;
    if (!sa.force_all && d.flag[(size_t)sa.par * sa.R + r] == 0) return;
    __shared__ int cnt[kMaxCells + 1];
    __shared__ int part[kReorderThreads];
    const RepDev rd = d.rep[r];
    reorder_replica<P>(d, rd, r, sa.cur, cnt, part);
}

// blockIdx.y = replica (from r0), 256 / kListLanes atoms per block.
template <class P>
__global__ __launch_bounds__(256) void k_listrows(DevState d, StepArgs sa)
{
    constexpr int APB = 256 / kListLanes;  // atoms per block
    constexpr int W = list_lds_words<kListLanes>();
    __shared__ int lds[256 * W];
    const int r = sa.r0 + blockIdx.y;
    if (!sa.force_all && d.flag[(size_t)sa.par * sa.R + r] == 0) return;
    const RepDev rd = d.rep[r];
    const int i = blockIdx.x * APB + (int)(threadIdx.x / kListLanes);
    if ((int)blockIdx.x * APB >= rd.N) return;
    const typename P::pos_t* pos = P::pos(d, sa.cur) + rd.base;
    list_rows<P, kListLanes>(d, rd, pos, i, i < rd.N, (int)(threadIdx.x % kListLanes), sa.tpa, sa.M,
                             lds + threadIdx.x * W);
}

// Force + epilogue; the first block of each replica also marks the list of
// this parity consumed and the pending velocity factor applied.
template <class P, int MODE, int TPA>
__global__ __launch_bounds__(256) void k_force(DevState d, StepArgs sa)
{
    const int b = sa.blk_off + blockIdx.x;
    const int r = sa.tab.rep[b];
    if (r < 0) return;
    const RepDev rd = d.rep[r];
    const int a0 = sa.tab.a0[b];
    if (MODE != kQuery && a0 == 0 && threadIdx.x == 0) {
        d.flag[(size_t)sa.par * sa.R + r] = 0u;
        d.alpha[r] = 1.0;
    }
    const int ia = a0 + (int)(threadIdx.x / TPA);
    force_atom<P, MODE, TPA>(d, sa, rd, r, ia, (int)(threadIdx.x % TPA), ia < rd.N, sa.cur, sa.step, sa.par);
}

// Per-replica reductions at a stopped boundary: the potential energy
// (do_u) and the velocity rescale factor of the thermostat (do_svr).
template <class P>
__global__ __launch_bounds__(256) void k_energy(DevState d, StepArgs sa)
{
    __shared__ double part[512];
    const int r = sa.r0 + blockIdx.x;
    const RepDev rd = d.rep[r];
    if (sa.do_u) energy_replica<P>(d, rd, r, part);
    if (sa.do_svr) svr_replica<P>(d, rd, r, sa.step, sa.seed, sa.svr_c, part);
}

// ---------------------------------------------------------------------------
// Exchange attempt k (Implementation section): ladder slots (j, j+1) with
// j = k mod 2 are paired -- or, with non-nearest-neighbour exchanges, slots
// (j, j+d) at the attempt's distance d (j >= o = (k mod 2) d with
// floor((j - o)/d) even); for the replicas a, b holding them
// D = (1/T_j - 1/T_{j+1}) (U_a - U_b); the 53-bit uniform of the lower
// replica id decides: accept iff D >= 0 or u < exp(D).  Accepted pairs swap
// slots; each swapped replica's pending velocity factor is multiplied by
// sqrt(T_new/T_old) and it takes the noise amplitude of its new temperature.
__device__ void exchange_body(const double* U, const double* Tl, int32_t* slot, int R, int64_t k, uint64_t seed,
                              int max_distance, double* alpha, double* c2, double c1sq, int64_t* att, int64_t* acc,
                              XRec* log, int64_t* log_count, int64_t log_cap, const int64_t* steps,
                              int64_t step_all, int32_t master, uint8_t* dec)
{
    __shared__ int rep[4096];
    __shared__ int64_t lbase;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int r = tid; r < R; r += nt) rep[slot[r]] = r;
    if (tid == 0) lbase = log_count ? *log_count : 0;
    __syncthreads();
    // pairs (j, j + dk): j >= o with floor((j - o) / dk) even; the p-th
    // such j is o + 2 dk (p / dk) + p mod dk
    const int dk = pattern_distance(seed, k, max_distance);
    const int o = (int)(k & 1) * dk;
    const int span = R - dk - o;
    const int npairs = span <= 0 ? 0 : (span / (2 * dk)) * dk + min(span % (2 * dk), dk);
    for (int p = tid; p < npairs; p += nt) {
        const int j = o + 2 * dk * (p / dk) + p % dk, h = j + dk;
        const int a = rep[j], b = rep[h];
        const double Ta = Tl[j], Tb = Tl[h];
        const double delta = (1.0 / Ta - 1.0 / Tb) * (U[a] - U[b]);
        const double u = uniform53(seed, k, a < b ? a : b);
        const int ok = (delta >= 0.0 || u < exp(delta)) ? 1 : 0;
        if (dec) dec[j] = (uint8_t)ok;
        if (att) att[j] += 1;
        if (acc) acc[j] += ok;
        if (log) {
            XRec rec;
            rec.attempt = k;
            rec.master = master;
            rec.slot_lo = j;
            rec.rep_a = a;
            rec.rep_b = b;
            rec.step_a = step_all >= 0 ? step_all : steps[a];
            rec.step_b = step_all >= 0 ? step_all : steps[b];
            rec.U_a = U[a];
            rec.U_b = U[b];
            rec.T_a = Ta;
            rec.T_b = Tb;
            rec.u = u;
            rec.accepted = ok;
            rec.slot_hi = h;
            log[(lbase + p) % log_cap] = rec;
        }
        if (ok) {
            slot[a] = h;
            slot[b] = j;
            if (alpha) {  // factors of consecutive exchanges compose
                alpha[a] *= sqrt(Tb / Ta);
                alpha[b] *= sqrt(Ta / Tb);
            }
            if (c2) {
                c2[a] = sqrt((1.0 - c1sq) * Tb);
                c2[b] = sqrt((1.0 - c1sq) * Ta);
            }
        }
    }
    __syncthreads();
    if (tid == 0 && log_count) *log_count = lbase + npairs;
}

__global__ __launch_bounds__(1024) void k_exchange(DevState d, int R, int64_t k, uint64_t seed, double c1sq,
                                                   int32_t master, int64_t log_cap, int64_t step_all, int maxd)
{
    exchange_body(d.U, d.Tl, d.slot, R, k, seed, maxd, d.alpha, d.c2, c1sq, d.attempts, d.accepts, d.log,
                  d.log_count, log_cap, d.steps, step_all, master, nullptr);
}

__global__ __launch_bounds__(1024) void k_test_exchange(const double* U, const double* Tl, int32_t* slot, int R,
                                                        uint64_t seed, int64_t k, int maxd, uint8_t* dec)
{
    for (int j = threadIdx.x; j < R - 1; j += blockDim.x) dec[j] = 255;
    __syncthreads();
    exchange_body(U, Tl, slot, R, k, seed, maxd, nullptr, nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, 1,
                  nullptr, 0, -1, dec);
}

__global__ void k_test_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, int n, uint32_t* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 w = philox10(make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]), k0, k1);
    out[4 * i] = w.x;
    out[4 * i + 1] = w.y;
    out[4 * i + 2] = w.z;
    out[4 * i + 3] = w.w;
}

__global__ void k_test_normals(int fp64, uint64_t seed, const uint32_t* ctr, int n, double* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 w = draw(seed, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    if (fp64) {
        double z0, z1, z2;
        normals3d(w, z0, z1, z2);
        out[3 * i] = z0;
        out[3 * i + 1] = z1;
        out[3 * i + 2] = z2;
    } else {
        float z0, z1, z2;
        normals3f(w, z0, z1, z2);
        out[3 * i] = z0;
        out[3 * i + 1] = z1;
        out[3 * i + 2] = z2;
    }
}

__global__ void k_clear_flags(DevState d, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d.flag[i] = 0u;
}

__global__ void k_set_steps(DevState d, int R, int64_t step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < R) d.steps[i] = step;
}

// ---------------------------------------------------------------------------
// Launch wrappers.
template <class P>
static hipError_t start_t(const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL(k_start<P>, dim3(nblk), dim3(sa.block), 0, st, d, sa);
    return hipGetLastError();
}

hipError_t launch_start(bool fp64, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    return fp64 ? start_t<PF64>(d, sa, nblk, st) : start_t<PMixed>(d, sa, nblk, st);
}

hipError_t launch_reorder(bool fp64, const DevState& d, const StepArgs& sa, int nrep, hipStream_t st)
{
    if (nrep <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_reorder<PF64>, dim3(nrep), dim3(kReorderThreads), 0, st, d, sa);
    else
        hipLaunchKernelGGL(k_reorder<PMixed>, dim3(nrep), dim3(kReorderThreads), 0, st, d, sa);
    return hipGetLastError();
}

hipError_t launch_listbuild(bool fp64, const DevState& d, const StepArgs& sa, int nrep, int nmax, hipStream_t st)
{
    if (nrep <= 0) return hipSuccess;
    const int apb = 256 / kListLanes;
    const dim3 grid((nmax + apb - 1) / apb, nrep);
    if (fp64)
        hipLaunchKernelGGL(k_listrows<PF64>, grid, dim3(256), 0, st, d, sa);
    else
        hipLaunchKernelGGL(k_listrows<PMixed>, grid, dim3(256), 0, st, d, sa);
    return hipGetLastError();
}

template <class P, int MODE>
static hipError_t force_mode(const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    switch (sa.tpa) {
    case 1: hipLaunchKernelGGL((k_force<P, MODE, 1>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    case 2: hipLaunchKernelGGL((k_force<P, MODE, 2>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    case 4: hipLaunchKernelGGL((k_force<P, MODE, 4>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    case 8: hipLaunchKernelGGL((k_force<P, MODE, 8>), dim3(nblk), dim3(sa.block), 0, st, d, sa); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class P>
static hipError_t force_t(StepMode mode, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    switch (mode) {
    case kFused: return force_mode<P, kFused>(d, sa, nblk, st);
    case kStop: return force_mode<P, kStop>(d, sa, nblk, st);
    case kStopEnergy: return force_mode<P, kStopEnergy>(d, sa, nblk, st);
    case kQuery: return force_mode<P, kQuery>(d, sa, nblk, st);
    case kRefresh: return force_mode<P, kRefresh>(d, sa, nblk, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_force(bool fp64, StepMode mode, const DevState& d, const StepArgs& sa, int nblk, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    return fp64 ? force_t<PF64>(mode, d, sa, nblk, st) : force_t<PMixed>(mode, d, sa, nblk, st);
}

hipError_t launch_energy(bool fp64, const DevState& d, const StepArgs& sa, int nrep, hipStream_t st)
{
    if (nrep <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_energy<PF64>, dim3(nrep), dim3(256), 0, st, d, sa);
    else
        hipLaunchKernelGGL(k_energy<PMixed>, dim3(nrep), dim3(256), 0, st, d, sa);
    return hipGetLastError();
}

hipError_t launch_exchange(const DevState& d, int R, int64_t attempt, uint64_t seed, double c1sq, int32_t master,
                           int64_t log_cap, int64_t step_all, int max_distance, hipStream_t st)
{
    hipLaunchKernelGGL(k_exchange, dim3(1), dim3(1024), 0, st, d, R, attempt, seed, c1sq, master, log_cap, step_all,
                       max_distance);
    return hipGetLastError();
}

hipError_t launch_clear_flags(const DevState& d, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_flags, dim3((n + 255) / 256), dim3(256), 0, st, d, n);
    return hipGetLastError();
}

hipError_t launch_set_steps(const DevState& d, int R, int64_t step, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_steps, dim3((R + 255) / 256), dim3(256), 0, st, d, R, step);
    return hipGetLastError();
}

hipError_t launch_test_exchange(const double* U, const double* Tl, int32_t* slot, int R, uint64_t seed,
                                int64_t attempt, int max_distance, uint8_t* dec, hipStream_t st)
{
    hipLaunchKernelGGL(k_test_exchange, dim3(1), dim3(1024), 0, st, U, Tl, slot, R, seed, attempt, max_distance, dec);
    return hipGetLastError();
}

hipError_t launch_test_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, int n, uint32_t* out,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_test_philox, dim3((n + 255) / 256), dim3(256), 0, st, ctr, key0, key1, n, out);
    return hipGetLastError();
}

hipError_t launch_test_normals(int fp64, uint64_t seed, const uint32_t* ctr, int n, double* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_test_normals, dim3((n + 255) / 256), dim3(256), 0, st, fp64, seed, ctr, n, out);
    return hipGetLastError();
}

}  // namespace re
