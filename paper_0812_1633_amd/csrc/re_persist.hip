// re_persist.hip -- the persistent engine: one launch advances every replica
// for a whole re_step call.
//
// Each replica is served by a team of workgroups (team_size >= 1; teams of
// one need no inter-workgroup synchronisation).  A team walks its replica
// through BAOAB steps on its own schedule -- list updates, force phases and
// exchange joins happen when that replica needs them -- so replicas
// progress at their own speed and may have taken different numbers of steps
// between exchange attempts (Implementation section: asynchronous
// iteration).  Team members synchronise through a counter barrier (agent-
// scope acquire; the release skips the L2 write-back when every member runs
// on one XCD); the leader (member 0) runs the reorder, the energy sum and
// the exchange protocol.
//
// Exchange protocol, attempt k (k0 = first attempt of the call):
//   gate     every replica has resolved attempt k-1 (the "done" counter
//            reached R (k - k0)) -- the master's blocking gather of the
//            temperatures in the paper;
//   pattern  slots entering attempt k are in slotbuf[k & 1]; ladder pairs
//            (j, j+1) with j = k mod 2;
//   post     U and join step into the mailbox of parity k & 1, then the
//            post counter (release);
//   wait     for the partner's post (acquire) -- the paper's blocking
//            receive of the (T, U, random) triplet;
//   decide   both partners evaluate the same Metropolis rule with the
//            Philox uniform of the lower replica id; the lower slot logs;
//   resolve  new slot into slotbuf[(k+1) & 1], velocity factor, done += 1.
// Triggers: synchronous mode joins at every multiple of N_x; asynchronous
// mode lets master m_k = k mod R trigger attempt k after N_x of its own
// steps since its previous attempt (the trigger counter), every other
// replica joining at its next step boundary after it sees the trigger;
// schedule mode joins at injected steps.  Every wait is bounded by the
// watchdog; a timeout raises the abort flag and every team exits.
#include "re_device.hpp"
#include <type_traits>

#include "re_persist.hpp"

namespace re {

__device__ __forceinline__ uint64_t clock100()
{
    return __builtin_amdgcn_s_memrealtime();  // 100 MHz constant clock
}

// Optional phase timers (built with RE_PHASE_TIMERS): thread 0 of every
// workgroup adds the 100 MHz ticks spent in each phase of k_persist to its
// own row; re_debug_phase_ticks copies the rows out and clears them.
#ifdef RE_PHASE_TIMERS
// phases 0..7 of the step loop; 8, 9: inside the exchange join, the wait
// at the gate and the wait for the partner's post; 10, 11: the leader's
// potential energy and velocity rescale at a stopped boundary
constexpr int kPhases = 12;
__device__ unsigned long long g_phase_ticks[1024 * kPhases];
#define PT_INIT() uint64_t pt_last = clock100()
#define PT_MARK(k)                                                  \
    do {                                                            \
        if (threadIdx.x == 0) {                                     \
            const uint64_t pt_now = clock100();                     \
            g_phase_ticks[blockIdx.x * kPhases + (k)] += pt_now - pt_last; \
            pt_last = pt_now;                                       \
        }                                                           \
    } while (0)
#else
#define PT_INIT() \
    do {          \
    } while (0)
#define PT_MARK(k) \
    do {           \
    } while (0)
#endif

// Copy f(src[k]), k < n, from global memory to LDS with the whole
// workgroup.  Every thread issues its loads of up to K elements before its
// first store, so a copy of K * blockDim elements waits for one memory
// latency, not K (load indices are clamped into the array, so no load
// depends on a branch).
template <int K, class D, class S, class F>
__device__ __forceinline__ void stage_to_lds(D* dst, const S* src, int n, F f)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int base = 0; base < n; base += K * nt) {
        S v[K];
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = src[min(base + tid + j * nt, n - 1)];
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (base + tid + j * nt < n) dst[base + tid + j * nt] = f(v[j]);
    }
}

// Bounded waiting (thread 0 of a workgroup).  The watchdog counts time
// without progress: any completed force phase anywhere (the heartbeat)
// restarts it.  On expiry the abort flag is raised.
struct Watch {
    uint64_t t0, beat;
};

__device__ __forceinline__ Watch watch_start(const PersistArgs& pa)
{
    return Watch{clock100(), __hip_atomic_load(pa.st.beat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}

// false: give up (abort raised or seen)
__device__ __forceinline__ bool watch_tick(const PersistArgs& pa, Watch& w)
{
    if (__hip_atomic_load(pa.st.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    const uint64_t b = __hip_atomic_load(pa.st.beat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t now = clock100();
    if (b != w.beat) {
        w.beat = b;
        w.t0 = now;
    } else if (now - w.t0 > pa.timeout) {
        atomicOr(pa.st.abort, 1u);
        atomicOr(pa.st.err, kErrTimeout);
        return false;
    }
    return true;
}

// thread 0 of a workgroup: spin until *p >= v (agent scope)
__device__ bool wait_ge_u64(const PersistArgs& pa, const uint64_t* p, uint64_t v)
{
    Watch w = watch_start(pa);
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
        __builtin_amdgcn_s_sleep(2);
        if (!watch_tick(pa, w)) return false;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

__device__ bool wait_ge_i64(const PersistArgs& pa, const int64_t* p, int64_t v)
{
    return wait_ge_u64(pa, reinterpret_cast<const uint64_t*>(p), (uint64_t)v);
}

// Team barrier: a counter per team.  Mode agent (any placement):
// agent-scope release/acquire around the counter, i.e. write-back of this
// XCD's L2 and invalidation of L1 and L2 for lines of other XCDs.  Mode
// one-XCD (every workgroup of the team reported the same XCC, so the team
// shares one L2): release is each wave waiting for its own stores to
// complete at the L2 (s_waitcnt 0) before the workgroup barrier -- no L2
// write-back -- and acquire stays agent-scope.  Returns false when the run
// is being aborted.
__device__ bool team_sync(const PersistArgs& pa, unsigned* ctr, unsigned& epoch, int t, bool one_xcd, int* s_ok)
{
    if (one_xcd) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        if (t > 1) {
            ++epoch;
            if (one_xcd)
                __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned tgt = epoch * (unsigned)t;
            Watch w = watch_start(pa);
            while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < tgt) {
                __builtin_amdgcn_s_sleep(1);
                if (!watch_tick(pa, w)) {
                    ok = 0;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        } else if (__hip_atomic_load(pa.st.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = 0;
        }
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Test hook: after a team barrier, one workgroup in four, picked by a hash
// of (workgroup, step, site), pauses for a pseudo-random part of
// delay_ticks (off when 0).  Results must not depend on it.
__device__ __forceinline__ void maybe_pause(const PersistArgs& pa, int b, int64_t s, int site)
{
    if (pa.delay_ticks == 0) return;
    uint32_t h = (uint32_t)b * 0x9E3779B1u ^ (uint32_t)s * 0x85EBCA77u ^ (uint32_t)site * 0xC2B2AE3Du;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    if ((h & 3u) != 0) return;
    if (threadIdx.x == 0) {
        const uint64_t t0 = clock100();
        const uint64_t len = (uint64_t)pa.delay_ticks * ((h >> 2) & 15u) / 15u;
        while (clock100() - t0 < len) __builtin_amdgcn_s_sleep(8);
    }
    __syncthreads();
}

// The exchange join of replica r at its boundary s (energy U) for attempt k,
// run by the whole leader workgroup.  Returns false on abort.
__device__ bool exchange_join(const DevState& d, const PersistArgs& pa, const CallParams& cp, int r, int64_t k,
                              int64_t s, double U, int* sh)
{
    const PersistState& ps = pa.st;
    const int R = pa.sa.R;
    const int p = (int)(k & 1);
    if (threadIdx.x == 0) {
#ifdef RE_PHASE_TIMERS
        const uint64_t tg0 = clock100();
#endif
        int ok = wait_ge_u64(pa, ps.xdone, (uint64_t)R * (uint64_t)(k - cp.k0)) ? 1 : 0;
#ifdef RE_PHASE_TIMERS
        g_phase_ticks[blockIdx.x * kPhases + 8] += clock100() - tg0;
#endif
        if (ok && cp.mode == kModeAsync && (int)(k % R) == r) {
            // the master publishes the trigger of attempt k
            __hip_atomic_fetch_max(ps.trig, (uint64_t)(k + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        sh[0] = ok;
        sh[1] = -1;
    }
    __syncthreads();
    if (!sh[0]) return false;
    const int32_t* sb = ps.slotbuf + (size_t)p * R;
    const int jme = sb[r];
    // partner slot: (j, j + dk) pairs with j >= o, floor((j - o)/dk) even
    const int dk = pattern_distance(pa.sa.seed, k, pa.xmaxd);
    const int o = p * dk;
    int jp = -1;
    if (jme >= o) {
        if ((((jme - o) / dk) & 1) == 0) {
            if (jme + dk < R) jp = jme + dk;
        } else {
            jp = jme - dk;
        }
    }
    if (jp >= 0)
        for (int q = threadIdx.x; q < R; q += blockDim.x)
            if (sb[q] == jp) sh[1] = q;
    __syncthreads();
    int ok = 1;
    if (threadIdx.x == 0) {
        const int q = sh[1];
        ps.upost[(size_t)p * R + r] = U;
        ps.spost[(size_t)p * R + r] = s;
        __hip_atomic_store(ps.post + r, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int newslot = jme;
        if (q >= 0) {
            // what does not depend on the partner's post is read or drawn
            // before the wait for it
            const int jlo = jme < jp ? jme : jp, jhi = jme < jp ? jp : jme;
            const int a = jme < jp ? r : q, b = jme < jp ? q : r;
            const double Ta = d.Tl[jlo], Tb = d.Tl[jhi];
            const double u = uniform53(pa.sa.seed, k, a < b ? a : b);
            const double apend = d.alpha[r];
#ifdef RE_PHASE_TIMERS
            const uint64_t tp0 = clock100();
#endif
            ok = wait_ge_i64(pa, ps.post + q, k + 1) ? 1 : 0;
#ifdef RE_PHASE_TIMERS
            g_phase_ticks[blockIdx.x * kPhases + 9] += clock100() - tp0;
#endif
            if (ok) {
                const double Uq = ps.upost[(size_t)p * R + q];
                const int64_t sq = ps.spost[(size_t)p * R + q];
                const double Ua = jme < jp ? U : Uq, Ub = jme < jp ? Uq : U;
                const double delta = (1.0 / Ta - 1.0 / Tb) * (Ua - Ub);
                const int acc = (delta >= 0.0 || u < exp(delta)) ? 1 : 0;
                if (jme == jlo) {
                    atomicAdd((unsigned long long*)&d.attempts[jlo], 1ull);
                    if (acc) atomicAdd((unsigned long long*)&d.accepts[jlo], 1ull);
                    const int64_t li = (int64_t)atomicAdd((unsigned long long*)d.log_count, 1ull);
                    XRec rec;
                    rec.attempt = k;
                    rec.master = cp.mode == kModeAsync ? (int32_t)(k % R) : -1;
                    rec.slot_lo = jlo;
                    rec.rep_a = a;
                    rec.rep_b = b;
                    rec.step_a = jme < jp ? s : sq;
                    rec.step_b = jme < jp ? sq : s;
                    rec.U_a = Ua;
                    rec.U_b = Ub;
                    rec.T_a = Ta;
                    rec.T_b = Tb;
                    rec.u = u;
                    rec.accepted = acc;
                    rec.slot_hi = jhi;
                    d.log[li % pa.log_cap] = rec;
                }
                if (acc) {
                    newslot = jp;
                    const double Tme = jme == jlo ? Ta : Tb, Tp = jme == jlo ? Tb : Ta;
                    d.alpha[r] = apend * sqrt(Tp / Tme);
                    d.c2[r] = sqrt((1.0 - pa.c1sq) * Tp);
                    ps.apend[r] = 1;
                }
            }
        }
        if (ok) {
            ps.slotbuf[(size_t)(p ^ 1) * R + r] = newslot;
            d.slot[r] = newslot;
            __hip_atomic_fetch_add(ps.xdone, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        sh[0] = ok;
    }
    __syncthreads();
    return sh[0] != 0;
}

// control word of a boundary: bit 0 stop at the next force phase, bit 1 join
// at that boundary, bit 2 leave the run here, bit 3 the stop needs the
// potential energy (a stop for the velocity rescale alone does not)
constexpr int kCtlStop = 1, kCtlJoin = 2, kCtlExit = 4, kCtlEnergy = 8;
// a step that stops only for the velocity rescale: its force phase stops,
// and the rescale and the next step's first half follow inside the step loop
constexpr int kCtlSVR = 16;

// SVR: compiled for the stochastic velocity rescale (whose steps end inside
// the step loop, see kCtlSVR); the Langevin form carries none of that code.
template <class P, int TPA, bool SVR>
__global__ __launch_bounds__(1024) void k_persist(DevState d, PersistArgs pa)
{
    // reorder counts; between reorders the list-build tables, then (when
    // they fit) copies of the replica's list keys and cell starts during a
    // list build, of its positions during the force sums
    __shared__ int cnt[kPersistLdsWords];
    using key_t = typename P::key_t;
    constexpr int kTabWords = 1024 * list_lds_words<kListLanes>();
    constexpr int kPosWords = (int)(sizeof(typename P::pos_t) / sizeof(int));
    constexpr int kKeyWords = (int)(sizeof(key_t) / sizeof(int));
    // list keys that are the positions themselves stay for the force sums
    constexpr bool kKeyIsPos = std::is_same<key_t, typename P::pos_t>::value;
    // positions staged per thread and round: 64 bytes of registers
    constexpr int kStageK = (int)(64 / sizeof(typename P::pos_t));
    static_assert(kTabWords <= kMaxCells + 1 && kMaxCells + 1 <= kPersistLdsWords, "LDS array too small");
    __shared__ int part[1024];
    __shared__ double dpart[kRedLds];
    __shared__ double r1tab[64];
    __shared__ long long r1lo;  // first boundary of r1tab (-1: none)
    __shared__ int sh[4];
    __shared__ int lr_next;  // list build: next batch of atoms to hand out
    if (threadIdx.x == 0) {
        lr_next = 0;
        r1lo = -1;
    }
    const PersistState& ps = pa.st;
    const CallParams& cp = *pa.call;
    const int b = blockIdx.x;
    const int r = pa.team_rep[b];
    if (r < 0) return;
    const int m = pa.team_mem[b], t = pa.team_size[b];
    unsigned* ctr = pa.bar + 64 * (size_t)pa.team_id[b];
    const bool leader = m == 0;
    const RepDev rd = d.rep[r];
    const int R = pa.sa.R;
    const int chunk = (rd.N + t - 1) / t;
    const int i0 = min(rd.N, m * chunk), i1 = min(rd.N, i0 + chunk);
    const int tid = threadIdx.x, nt = blockDim.x;
    unsigned epoch = 0;
    // which XCDs does the team run on?  Every member reports its XCC before
    // a first agent-scope barrier; one XCC for all allows the one-XCD barrier
    bool one_xcd = false;
    if (t > 1) {
        if (tid == 0) {
            const unsigned xcc = __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 0xFu;  // HW_REG_XCC_ID
            atomicOr(ps.xmask + pa.team_id[b], 1u << xcc);
        }
        if (!team_sync(pa, ctr, epoch, t, false, &sh[3])) return;
        const unsigned msk =
            __hip_atomic_load(ps.xmask + pa.team_id[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        one_xcd = pa.bar_mode == 1 && __builtin_popcount(msk) == 1;
    }
    // per-replica state, identical in every member
    int64_t s = d.steps[r];
    const int cur0 = cp.cur0;
    int cur = cur0;
    int64_t knext = ps.katt[r];
    int64_t jprev = ps.jprev[r];
    int64_t asched = 0;  // next scheduled attempt (schedule mode)
    int64_t target = cp.mode == kModeSchedule ? 0 : s + cp.n;
    bool join_pending = false;
    bool parked = false;
    bool reached = false;  // asynchronous mode: this replica reached its target
    double Ucur = d.U[r];  // potential energy at the last stop (thread 0's is used)
    // R1 of the velocity rescale at boundary sn, from a table of the 64
    // boundaries from r1lo on that the first wave fills (a normal per lane)
    // when sn is not in it; called by the whole workgroup
    auto svr_r1 = [&](int64_t sn) -> double {
        const long long lo = r1lo;
        if (lo < 0 || sn < lo || sn >= lo + 64) {
            if (tid < 64) r1tab[tid] = svr_normal(pa.sa.seed, sn + tid, r);
            __syncthreads();
            if (tid == 0) r1lo = sn;
            __syncthreads();
            return r1tab[0];
        }
        return r1tab[sn - lo];
    };
    // synchronous form: the next multiple of N_x not below the boundaries
    // planned so far (advanced as they pass; no 64-bit division per step)
    int64_t xnext = (s + pa.Nx - 1) / pa.Nx * pa.Nx;

    // plan for the force phase that ends at boundary sn (leader only;
    // boundaries are planned in increasing order)
    auto plan = [&](int64_t sn) -> int {
        int c = 0;
        if (cp.mode == kModeSync) {
            while (xnext < sn) xnext += pa.Nx;
            if (sn == xnext) c |= kCtlStop | kCtlJoin;
            if (sn >= target) c |= kCtlStop;
        } else if (cp.mode == kModeSchedule) {
            if (asched < cp.A && sn == cp.sched[asched * R + r]) c |= kCtlStop | kCtlJoin;
        } else {
            const bool master = (int)(knext % R) == r;
            if (master && sn == jprev + pa.Nx) c |= kCtlStop | kCtlJoin;
            if (!master &&
                __hip_atomic_load(ps.trig, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > (uint64_t)knext)
                c |= kCtlStop | kCtlJoin;
            // stop on reaching the target, and once every replica has
            // reached its own (then this one parks)
            if (!reached && sn >= target) c |= kCtlStop;
            if (reached && __hip_atomic_load(ps.reach, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)R)
                c |= kCtlStop;
        }
        // every stop for an exchange or the end of the call computes U (in
        // the asynchronous form every stop: a replica may find at the
        // boundary that it parks, and then joins attempts with its U)
        if ((c & kCtlStop) || cp.mode == kModeAsync) c |= kCtlEnergy;
        // the velocity rescale needs the velocities of every atom at the end of
        // every step: the force phase stops (a step that stops for nothing
        // else is marked kCtlSVR and goes on inside the step loop)
        if constexpr (SVR) {
            if (!(c & kCtlStop)) c |= kCtlStop | kCtlSVR;
        } else if (pa.sa.thermo == kThermoSVR) {
            c |= kCtlStop;
        }
        return c;
    };

    bool ok = true;
    int ctl = 0;
    PT_INIT();
    while (ok) {
        // ---- at a stopped boundary s
        if (leader) {
            if (join_pending) {
                ok = exchange_join(d, pa, cp, r, knext, s, Ucur, sh);
                knext += 1;
                jprev = s;
                if (cp.mode == kModeSchedule) asched += 1;
                join_pending = false;
            }
            int c = 0;
            if (ok) {
                bool done;
                if (cp.mode == kModeSync) {
                    done = s >= target;
                } else if (cp.mode == kModeSchedule) {
                    done = asched >= cp.A;
                } else {
                    // asynchronous: a replica past its target keeps stepping
                    // (and exchanging) until every replica has reached its
                    // own, so that no replica idles while others catch up
                    if (!reached && s >= target) {
                        reached = true;
                        if (tid == 0)
                            __hip_atomic_fetch_add(ps.reach, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (tid == 0)
                        sh[2] = reached && __hip_atomic_load(ps.reach, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)R;
                    __syncthreads();
                    done = sh[2] != 0;
                    __syncthreads();
                }
                if (done && cp.mode == kModeAsync) {
                    // parked: take part in attempts triggered by others until
                    // every replica is parked and no attempt is in flight
                    if (!parked && tid == 0) __hip_atomic_fetch_add(ps.parked, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    parked = true;
                    Watch w{};
                    if (tid == 0) w = watch_start(pa);
                    while (ok) {
                        if (tid == 0) {
                            const uint64_t tr = __hip_atomic_load(ps.trig, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                            const uint64_t pk = __hip_atomic_load(ps.parked, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                            const uint64_t xd = __hip_atomic_load(ps.xdone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                            int act = 0;
                            if (tr > (uint64_t)knext)
                                act = 1;  // join
                            else if (pk == (uint64_t)R && xd == (uint64_t)R * (tr - (uint64_t)cp.k0))
                                act = 2;  // everyone parked, nothing in flight
                            else if (!watch_tick(pa, w))
                                act = 3;
                            else
                                __builtin_amdgcn_s_sleep(4);
                            sh[2] = act;
                        }
                        __syncthreads();
                        const int act = sh[2];
                        __syncthreads();
                        if (act == 1) {
                            ok = exchange_join(d, pa, cp, r, knext, s, Ucur, sh);
                            knext += 1;
                            jprev = s;
                        } else if (act == 2) {
                            break;
                        } else if (act == 3) {
                            ok = false;
                        }
                    }
                    c = kCtlExit;
                } else if (done) {
                    c = kCtlExit;
                } else {
                    c = plan(s + 1);
                }
            }
            if (!ok) c = kCtlExit;
            if (tid == 0) ps.ctl[(size_t)((s + 1) & 1) * R + r] = c;
        }
        if (!team_sync(pa, ctr, epoch, t, one_xcd, &sh[3])) {
            ok = false;
            break;
        }
        maybe_pause(pa, b, s, 0);
        ctl = __hip_atomic_load(ps.ctl + (size_t)((s + 1) & 1) * R + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        PT_MARK(0);
        if (ctl & kCtlExit) break;
        // ---- first half of step s -> s+1
        {
            const bool apply = __hip_atomic_load(ps.apend + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            for (int i = i0 + tid; i < i1; i += nt) start_atom<P>(d, pa.sa, rd, r, i, cur, s, apply);
        }
        if (!team_sync(pa, ctr, epoch, t, one_xcd, &sh[3])) {
            ok = false;
            break;
        }
        maybe_pause(pa, b, s, 1);
        if (leader && tid == 0) {
            d.alpha[r] = 1.0;
            ps.apend[r] = 0;
        }
        PT_MARK(1);
        // ---- steps that end at a fused boundary loop here
        for (;;) {
            const int par = (int)((s + 1) & 1);
            const bool rebuild = __hip_atomic_load(d.flag + (size_t)par * R + r, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT) == rebuild_tag(s + 1);
            bool staged = false;  // this step's positions already copied to LDS
            if (rebuild) {
                if (leader) reorder_replica<P>(d, rd, r, cur, cnt, part);
                if (!team_sync(pa, ctr, epoch, t, one_xcd, &sh[3])) {
                    ok = false;
                    break;
                }
                maybe_pause(pa, b, s, 2);
                PT_MARK(2);
                const typename P::pos_t* pos = P::pos(d, cur) + rd.base;
                const int32_t* cs = d.cell_start + rd.cell_base;
                const int ncs = rd.ncell * rd.ncell * rd.ncell + 1;
                const bool keys_lds = kTabWords + kKeyWords * rd.N + ncs <= kPersistLdsWords;
                // batches of one wave's atoms go to the waves as they finish
                // (the lists do not depend on which wave builds them)
                constexpr int kApw = 64 / kListLanes;  // atoms per wave
                const int nbatch = (i1 - i0 + kApw - 1) / kApw;
                auto build = [&](const auto* keys, const int32_t* csp) __attribute__((always_inline)) {
                    for (;;) {
                        int bi = 0;
                        if ((tid & 63) == 0) bi = atomicAdd(&lr_next, 1);
                        bi = __shfl(bi, 0);
                        if (bi >= nbatch) break;
                        const int i = i0 + bi * kApw + (tid & 63) / kListLanes;
                        list_rows<P, kListLanes>(d, rd, pos, keys, csp, i, i < i1, tid % kListLanes, rd.tpa,
                                                 pa.sa.M, cnt + tid * list_lds_words<kListLanes>());
                    }
                };
                if (keys_lds) {
                    // the candidates' keys and the cell starts from LDS
                    key_t* lkey = reinterpret_cast<key_t*>(cnt + kTabWords);
                    int32_t* lcs = cnt + kTabWords + kKeyWords * rd.N;
                    stage_to_lds<kStageK>(lkey, pos, rd.N,
                                          [](const typename P::pos_t& p) { return P::list_key(p); });
                    stage_to_lds<4>(lcs, cs, ncs, [](int c) { return c; });
                    __syncthreads();
                    build((const key_t*)lkey, (const int32_t*)lcs);
                    staged = kKeyIsPos;
                } else {
                    build(pos, cs);
                }
                // every workgroup builds the lists of its own atoms and then
                // computes their forces: a workgroup barrier orders the two
                // (and ends the batch counter's use before its reset; its next
                // use follows further workgroup barriers)
                __syncthreads();
                if (tid == 0) lr_next = 0;
                PT_MARK(3);
            }
            const bool stop = (ctl & kCtlStop) != 0;
            const bool with_u = (ctl & kCtlEnergy) != 0;
            // the force sums read the replica's positions from an LDS copy
            // when it fits (a gather of 64 lanes from LDS instead of up to 64
            // L1 lines); the list build may have made it already
            // (the mixed form's copy starts at the array's first word, so that
            // a neighbour's LDS address is its list word itself, with no base
            // to add; the stash of the force sums follows it.  The FP64 form
            // keeps the copy where the list build left its keys.)
            const typename P::pos_t* gpos = P::pos(d, cur) + rd.base;
            // lanes per atom: the kernel's, or (TPA = 0) this replica's
            const int tpa_r = TPA ? TPA : rd.tpa;
            const int apb = nt / tpa_r;
            constexpr int kPosAt = kKeyIsPos ? kTabWords : 0;
            const int stash_words =
                tpa_r == 1 ? 0 : (int)((sizeof(typename P::vel_t) + sizeof(typename P::pos_t)) / sizeof(int)) * (1024 / tpa_r);
            const int pos_words = (kPosWords * rd.N + 7) & ~7;  // (32-byte aligned stash)
            const bool lds_pos = kKeyIsPos ? kTabWords + kPosWords * rd.N <= kPersistLdsWords
                                           : stash_words + pos_words <= kPersistLdsWords;
            const int stash_at = kKeyIsPos || !lds_pos ? 0 : pos_words;
            typename P::pos_t* lpos = reinterpret_cast<typename P::pos_t*>(cnt + kPosAt);
            if (lds_pos && !staged) {
                stage_to_lds<kStageK>(lpos, gpos, rd.N, [](const typename P::pos_t& p) { return p; });
                __syncthreads();
            }
            // with TPA > 1 the sums of a pass go through LDS so that the
            // epilogues run one atom per thread (in the lanes of the atom's
            // group all but one would idle); LDS free between list builds
            // (the stash takes the sums of G passes, and the epilogues of a
            // group run together: with the positions in LDS one pass per group,
            // else TL passes, so that every thread of the workgroup has an
            // epilogue atom instead of one in TL)
            auto force_pass = [&](auto mode, auto lanes, auto group, const typename P::pos_t* fpos, int a0,
                                  int a1) __attribute__((always_inline)) {
                constexpr int M = decltype(mode)::value;
                constexpr int TL = decltype(lanes)::value;
                constexpr int G = decltype(group)::value;
                using real = typename P::real;
                using real4 = typename P::vel_t;
                real4* lf = reinterpret_cast<real4*>(cnt + stash_at);
                typename P::pos_t* lp = reinterpret_cast<typename P::pos_t*>(lf + G * apb);
                for (int base = a0; base < a1; base += G * apb) {
                    if constexpr (TL == 1) {
                        const int ia = base + tid;
                        typename P::pos_t pi;
                        real fx, fy, fz, e;
                        force_sum<P, M, TL>(d, pa.sa, rd, fpos, ia, 0, ia < a1, pi, fx, fy, fz, e);
                        if (ia < a1) force_epilogue<P, M>(d, pa.sa, rd, r, ia, cur, s + 1, par, pi, fx, fy, fz, e);
                    } else {
                        for (int g = 0; g < G; ++g) {
                            const int ia = base + g * apb + tid / TL;
                            typename P::pos_t pi;
                            real fx, fy, fz, e;
                            force_sum<P, M, TL>(d, pa.sa, rd, fpos, ia, tid % TL, ia < a1, pi, fx, fy, fz, e);
                            if (tid % TL == 0 && ia < a1) {
                                real4 f;
                                f.x = fx;
                                f.y = fy;
                                f.z = fz;
                                f.w = e;
                                lf[g * apb + tid / TL] = f;
                                lp[g * apb + tid / TL] = pi;
                            }
                        }
                        // the velocity and x_ref of this thread's epilogue atom
                        // are loaded before the barrier, so that their latency
                        // overlaps the wait for the other waves' sums
                        const int ja = base + tid;
                        const bool epi = tid < G * apb && ja < a1;
                        real4 v0{};
                        typename P::pos_t xr0{};
                        if (epi) {
                            if constexpr (M != kQuery) v0 = P::vel(d)[rd.base + ja];
                            if constexpr (M == kFused) xr0 = P::xref(d)[rd.base + ja];
                        }
                        __syncthreads();
                        if (epi) {
                            const real4 f = lf[tid];
                            force_epilogue_v<P, M>(d, pa.sa, rd, r, ja, cur, s + 1, par, lp[tid], f.x, f.y, f.z, f.w,
                                                   v0, xr0);
                        }
                        if (base + G * apb < a1) __syncthreads();
                    }
                }
            };
            static_assert(2 * 1024 * sizeof(double4) <= sizeof(int) * kPersistLdsWords, "force stash exceeds LDS");
            // (separate calls for each position source, so that each inlined
            // copy knows its address space)
            auto run_lanes = [&](auto mode, auto lanes) __attribute__((always_inline)) {
                if (lds_pos)
                    force_pass(mode, lanes, std::integral_constant<int, 1>{}, lpos, i0, i1);
                else
                    force_pass(mode, lanes, lanes, gpos, i0, i1);
            };
            auto run = [&](auto mode) __attribute__((always_inline)) {
                if constexpr (TPA != 0) {
                    run_lanes(mode, std::integral_constant<int, TPA>{});
                } else {
                    switch (rd.tpa) {
                    case 1: run_lanes(mode, std::integral_constant<int, 1>{}); break;
                    case 2: run_lanes(mode, std::integral_constant<int, 2>{}); break;
                    case 4: run_lanes(mode, std::integral_constant<int, 4>{}); break;
                    default: run_lanes(mode, std::integral_constant<int, 8>{}); break;
                    }
                }
            };
            if (!stop)
                run(std::integral_constant<int, kFused>{});
            else if (with_u)
                run(std::integral_constant<int, kStopEnergy>{});
            else
                run(std::integral_constant<int, kStop>{});
            if (leader && !stop && tid == 0) ps.ctl[(size_t)((s + 2) & 1) * R + r] = plan(s + 2);
            PT_MARK(4);
#ifdef RE_PHASE_TIMERS
            __syncthreads();  // (timers: the workgroup's last wave apart from the team barrier)
            PT_MARK(7);
#endif
            if (!team_sync(pa, ctr, epoch, t, one_xcd, &sh[3])) {
                ok = false;
                break;
            }
            maybe_pause(pa, b, s, 3);
            PT_MARK(5);
            if (leader && tid == 0) __hip_atomic_fetch_add(ps.beat, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s += 1;
            if constexpr (SVR) {
            if (stop && (ctl & kCtlSVR)) {
                // the velocity rescale without leaving the step loop: every
                // member computes the factor (the same bits in each), then the
                // first half of the next step for its own atoms with the
                // pending factor (1 between exchanges) times it applied
                const double apend = d.alpha[r];  // (loaded before the reduction's barriers)
                const double R1 = svr_r1(s);
                const double fct = svr_factor<P>(d, rd, r, s, pa.sa.seed, pa.sa.svr_c, true, R1, dpart);
                const double a64 = apend * fct;
                for (int i = i0 + tid; i < i1; i += nt) start_atom_scaled<P>(d, pa.sa, rd, r, i, cur, s, a64);
                if (leader && tid == 0) ps.ctl[(size_t)((s + 1) & 1) * R + r] = plan(s + 1);
                if (!team_sync(pa, ctr, epoch, t, one_xcd, &sh[3])) {
                    ok = false;
                    break;
                }
                maybe_pause(pa, b, s, 6);
                PT_MARK(1);
                ctl = __hip_atomic_load(ps.ctl + (size_t)((s + 1) & 1) * R + r, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            }
            if (stop) {
                if (leader) {
                    if (with_u) Ucur = energy_replica<P>(d, rd, r, dpart);
                    PT_MARK(10);
                    if (pa.sa.thermo == kThermoSVR) {
                        const double R1 = svr_r1(s);
                        svr_replica<P>(d, rd, r, s, pa.sa.seed, pa.sa.svr_c, true, R1, dpart);
                        if (tid == 0) ps.apend[r] = 1;
                    }
                    PT_MARK(11);
                }
                PT_MARK(6);
                join_pending = (ctl & kCtlJoin) != 0;
                break;
            }
            cur ^= 1;
            ctl = __hip_atomic_load(ps.ctl + (size_t)((s + 1) & 1) * R + r, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // ---- leave at a stopped boundary: positions back into the call's buffer
    if (cur != cur0) {
        typename P::pos_t* src = P::pos(d, cur) + rd.base;
        typename P::pos_t* dst = P::pos(d, cur0) + rd.base;
        for (int i = i0 + tid; i < i1; i += nt) dst[i] = src[i];
    }
    if (leader && tid == 0) {
        d.steps[r] = s;
        ps.katt[r] = knext;
        ps.jprev[r] = jprev;
    }
}

// Reset of the per-call counters and the slots entering the first attempt.
__global__ void k_persist_prepare(DevState d, PersistArgs pa, int nteams)
{
    const PersistState& ps = pa.st;
    const CallParams& cp = *pa.call;
    const int R = pa.sa.R;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < R) {
        ps.slotbuf[(size_t)(cp.k0 & 1) * R + i] = d.slot[i];
        ps.katt[i] = cp.k0;
        if (cp.apply_alpha) ps.apend[i] = 1;
    }
    if (i < 64 * nteams) pa.bar[i] = 0u;
    if (i < nteams) ps.xmask[i] = 0u;
    if (i == 0) {
        *ps.xdone = 0ull;
        *ps.trig = (uint64_t)cp.k0;
        *ps.parked = 0u;
        *ps.reach = 0u;
        *ps.abort = 0u;
        *ps.err = 0u;
        *ps.beat = 0ull;
    }
}

template <class P, bool SVR>
static hipError_t persist_t(const DevState& d, const PersistArgs& pa, int nblk, hipStream_t st)
{
    switch (pa.sa.tpa) {
    case 0: hipLaunchKernelGGL((k_persist<P, 0, SVR>), dim3(nblk), dim3(1024), 0, st, d, pa); break;
    case 1: hipLaunchKernelGGL((k_persist<P, 1, SVR>), dim3(nblk), dim3(1024), 0, st, d, pa); break;
    case 2: hipLaunchKernelGGL((k_persist<P, 2, SVR>), dim3(nblk), dim3(1024), 0, st, d, pa); break;
    case 4: hipLaunchKernelGGL((k_persist<P, 4, SVR>), dim3(nblk), dim3(1024), 0, st, d, pa); break;
    case 8: hipLaunchKernelGGL((k_persist<P, 8, SVR>), dim3(nblk), dim3(1024), 0, st, d, pa); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_persist(bool fp64, const DevState& d, const PersistArgs& pa, int nblk, int nteams, hipStream_t st)
{
    const int n = std::max(pa.sa.R, 64 * nteams);
    hipLaunchKernelGGL(k_persist_prepare, dim3((n + 255) / 256), dim3(256), 0, st, d, pa, nteams);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool svr = pa.sa.thermo == kThermoSVR;
    if (fp64) return svr ? persist_t<PF64, true>(d, pa, nblk, st) : persist_t<PF64, false>(d, pa, nblk, st);
    if (pa.sa.n16) return svr ? persist_t<PMixed16, true>(d, pa, nblk, st) : persist_t<PMixed16, false>(d, pa, nblk, st);
    return svr ? persist_t<PMixed, true>(d, pa, nblk, st) : persist_t<PMixed, false>(d, pa, nblk, st);
}

#ifdef RE_PHASE_TIMERS
extern "C" int re_debug_phase_ticks(unsigned long long* out, int nblk)
{
    if (nblk < 0 || nblk > 1024) return -1;
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_ticks), sizeof(unsigned long long) * kPhases * nblk) !=
        hipSuccess)
        return -3;
    static unsigned long long zero[1024 * kPhases];
    return hipMemcpyToSymbol(HIP_SYMBOL(g_phase_ticks), zero, sizeof zero) == hipSuccess ? 0 : -3;
}
#endif

template <class P, bool SVR>
static const void* persist_kernel(int tpa)
{
    switch (tpa) {
    case 0: return (const void*)k_persist<P, 0, SVR>;
    case 1: return (const void*)k_persist<P, 1, SVR>;
    case 2: return (const void*)k_persist<P, 2, SVR>;
    case 4: return (const void*)k_persist<P, 4, SVR>;
    default: return (const void*)k_persist<P, 8, SVR>;
    }
}

hipError_t persist_occupancy(bool fp64, bool n16, int tpa, bool svr, int* blocks_per_cu)
{
    const void* f = fp64  ? (svr ? persist_kernel<PF64, true>(tpa) : persist_kernel<PF64, false>(tpa))
                    : n16 ? (svr ? persist_kernel<PMixed16, true>(tpa) : persist_kernel<PMixed16, false>(tpa))
                          : (svr ? persist_kernel<PMixed, true>(tpa) : persist_kernel<PMixed, false>(tpa));
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, 1024, 0);
}

}  // namespace re
