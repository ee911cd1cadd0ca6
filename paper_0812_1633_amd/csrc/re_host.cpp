// re_host.cpp -- host runtime and C ABI of the replica-exchange LJ engine.
//
// Owns the device arrays of a run, plans the launch tables, builds the
// initial state, drives the per-step launch sequences (batched lockstep and
// plain per-replica forms) and the persistent engine, and implements every
// entry point of include/re.h.
#include "re_internal.hpp"
#include "re_persist.hpp"
#include "re_tune.hpp"
#include "../../include/re.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

using namespace re;

// ---------------------------------------------------------------------------
// errors
static thread_local std::string g_noctx_error;

struct re_ctx {
    // run parameters
    int R = 0;
    int prec = RE_MIXED, form = RE_BATCHED, engine = RE_PERSISTENT, xmode = RE_SYNC;
    double rc = 0, skin = 0, dt = 0, gamma = 1.0;
    int thermo = 0;       // kThermoLangevin | kThermoSVR
    int xmaxd = 1;        // largest ladder distance of an exchange pair
    bool wide_reorder = false;  // lockstep: reorder large replicas with grid-wide passes
    int64_t total_atoms = 0;
    double svr_c = 1.0;   // exp(-dt / tau) of the velocity rescale
    int Nx = 1;
    uint64_t seed = 0;
    double ushift = 0, c1 = 0;
    double watchdog = 10.0;
    std::vector<int32_t> N;
    std::vector<int> tpa_r;  // force lanes per atom of each replica
    std::vector<double> rho, L, Tl;
    std::vector<RepDev> rep;
    // device
    DevState d{};
    LaunchCfg cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<void*> allocs;
    int64_t total_slots = 0;
    int total_cells = 0;
    int cells_max = 1;  // largest ncell^3 over the replicas
    int nmax = 0;       // largest replica
    // block tables: batched (XCD-interleaved over all replicas) and
    // contiguous (replica r at [start[r], start[r] + count[r]))
    BlockTable bt1{}, btF{}, ct1{}, ctF{};
    int nbt1 = 0, nbtF = 0;
    std::vector<int32_t> c1_start, c1_count, cF_start, cF_count;
    // lockstep state
    int cur = 0;
    int64_t step = 0;          // common step count (sync forms)
    int64_t next_attempt = 0;  // global attempt index
    int pending_alpha = 0;     // the next start kernel applies the exchange factor
    // persistent engine
    bool pers_ok = false;        // a team plan fits the device
    std::string pers_why;        // why not, when it does not
    PersistState ps{};
    CallParams* d_call = nullptr;
    CallParams* h_call = nullptr;  // pinned staging of the per-call parameters
    // status of a call, one contiguous block read back with one copy:
    // error bits (u32), list overflow (u32), next attempt per replica (R x
    // i64), steps per replica (R x i64); h_stat is its pinned host copy
    unsigned char* d_stat = nullptr;
    unsigned char* h_stat = nullptr;
    bool stat_valid = false;       // h_stat holds the state after the last persistent call
    std::vector<void*> pinned;     // pinned host allocations
    int64_t* d_sched = nullptr;
    int64_t sched_cap = 0;
    std::vector<int64_t> sched;  // pending injected schedule (A x R)
    int64_t sched_A = 0;
    int32_t *t_rep = nullptr, *t_mem = nullptr, *t_size = nullptr, *t_id = nullptr;
    unsigned* bar = nullptr;
    int pnblk = 0, pnteams = 0;
    std::vector<int> team_of;    // team size chosen per replica
    int team_opt = 0;            // explicit team size (0: automatic)
    bool balance = false;        // rebalance automatic teams from measured list-update rates
    std::vector<int64_t> plan_steps, plan_reb;  // steps and list updates at the last plan
    int rebalanced = 0;          // plans that changed a team since creation
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int bar_mode = 0;            // team barrier mode of the persistent engine
    int delay_us = 0;            // test hook: pauses after team barriers (persistent engine)
    // force-kernel timing with HIP events (re_profile)
    bool prof = false;
    std::vector<hipEvent_t> ev;  // pairs
    int ev_used = 0;
    double prof_ms = 0;
    int64_t prof_n = 0;
    std::string err;
};

static int fail(re_ctx* c, int code, const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_noctx_error = buf;
    return code;
}

int re::fail_noctx(int code, const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_noctx_error = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail((ctx), e_ == hipErrorOutOfMemory ? RE_ENOMEM : RE_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                             \
    } while (0)

template <class T>
static int dalloc(re_ctx* c, T** p, size_t n)
{
    void* q = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess) return fail(c, RE_ENOMEM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
    c->allocs.push_back(q);
    *p = (T*)q;
    return 0;
}

// ---------------------------------------------------------------------------
// Host Philox4x32-10 (SC'11 definition) for the initial state.
static void host_philox(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
    }
}

static double box_side(int32_t N, double rho)
{
    // (N/rho)^(1/3) rounded to a multiple of 2^-12: exact in FP32 and FP64,
    // and grid-aligned positions stay exact in FP64
    return std::nearbyint(std::cbrt((double)N / rho) * 4096.0) / 4096.0;
}

// FCC start with Maxwell-Boltzmann velocities (the initial state is not
// specified by the paper; see re_create in re.h for the definition).
static void init_replica(int32_t N, double L, double T, uint64_t seed, int r, std::vector<double>& x,
                         std::vector<double>& v)
{
    int n = 1;
    while (4 * n * n * n < N) ++n;
    const int M = 4 * n * n * n;
    std::vector<int> sites(N);
    if (M == N) {
        for (int i = 0; i < N; ++i) sites[i] = i;
    } else {
        std::vector<std::pair<uint32_t, int>> key(M);
        for (int m = 0; m < M; ++m) {
            uint32_t c[4] = {(uint32_t)m, 0u, (uint32_t)r, kPurposeVacancy};
            host_philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
            key[m] = {c[0], m};
        }
        std::partial_sort(key.begin(), key.begin() + N, key.end());
        for (int i = 0; i < N; ++i) sites[i] = key[i].second;
        std::sort(sites.begin(), sites.end());
    }
    static const double basis[4][3] = {{0, 0, 0}, {0.5, 0.5, 0}, {0.5, 0, 0.5}, {0, 0.5, 0.5}};
    const double a = L / n;
    x.resize(3 * (size_t)N);
    v.resize(3 * (size_t)N);
    for (int i = 0; i < N; ++i) {
        const int m = sites[i], b = m & 3, cell = m >> 2;
        const int iz = cell % n, iy = (cell / n) % n, ix = cell / (n * n);
        x[3 * i + 0] = (ix + basis[b][0] + 0.25) * a - 0.5 * L;
        x[3 * i + 1] = (iy + basis[b][1] + 0.25) * a - 0.5 * L;
        x[3 * i + 2] = (iz + basis[b][2] + 0.25) * a - 0.5 * L;
    }
    const double sT = std::sqrt(T), tau = 6.283185307179586476925286766559;
    double mean[3] = {0, 0, 0};
    for (int i = 0; i < N; ++i) {
        uint32_t c[4] = {(uint32_t)i, 0u, (uint32_t)r, kPurposeInitVel};
        host_philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        double u[4];
        for (int k = 0; k < 4; ++k) u[k] = ((double)c[k] + 0.5) * 0x1p-32;
        const double ra = std::sqrt(-2.0 * std::log(u[0])), rb = std::sqrt(-2.0 * std::log(u[2]));
        const double z[3] = {ra * std::cos(tau * u[1]), ra * std::sin(tau * u[1]), rb * std::cos(tau * u[3])};
        for (int k = 0; k < 3; ++k) {
            v[3 * i + k] = sT * z[k];
            mean[k] += v[3 * i + k];
        }
    }
    for (int k = 0; k < 3; ++k) mean[k] /= N;
    double s2 = 0;
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < 3; ++k) {
            v[3 * i + k] -= mean[k];
            s2 += v[3 * i + k] * v[3 * i + k];
        }
    const double f = std::sqrt((3.0 * N - 3.0) * T / s2);
    for (auto& q : v) q *= f;
}

// ---------------------------------------------------------------------------
// upload one replica's state in atom-id order (slot k holds atom k)
static int upload_replica(re_ctx* c, int r, const double* x, const double* v)
{
    const RepDev& rd = c->rep[r];
    const int N = rd.N;
    if (c->prec == RE_MIXED) {
        std::vector<int4> p(N);
        std::vector<float4> w(N);
        for (int i = 0; i < N; ++i) {
            int32_t q[3];
            for (int k = 0; k < 3; ++k) {
                const double xx = x[3 * i + k] - rd.L * std::floor(x[3 * i + k] / rd.L + 0.5);
                const int64_t g = (int64_t)std::nearbyint(xx * rd.inv_s);
                q[k] = (int32_t)(uint32_t)(uint64_t)g;
            }
            p[i] = make_int4(q[0], q[1], q[2], i);
            w[i] = make_float4((float)v[3 * i], (float)v[3 * i + 1], (float)v[3 * i + 2], 0.0f);
        }
        HIPCHK(c, hipMemcpyAsync(c->d.posi[c->cur] + rd.base, p.data(), N * sizeof(int4), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->d.velf + rd.base, w.data(), N * sizeof(float4), hipMemcpyHostToDevice, c->stream));
    } else {
        std::vector<double4> p(N), w(N);
        for (int i = 0; i < N; ++i) {
            double q[3];
            for (int k = 0; k < 3; ++k) q[k] = x[3 * i + k] - rd.L * std::floor((x[3 * i + k] + 0.5 * rd.L) / rd.L);
            p[i] = make_double4(q[0], q[1], q[2], (double)i);
            w[i] = make_double4(v[3 * i], v[3 * i + 1], v[3 * i + 2], 0.0);
        }
        HIPCHK(c, hipMemcpyAsync(c->d.posd[c->cur] + rd.base, p.data(), N * sizeof(double4), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->d.veld + rd.base, w.data(), N * sizeof(double4), hipMemcpyHostToDevice, c->stream));
    }
    // the host vectors die at return: wait for the copies
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
}

static StepArgs base_args(re_ctx* c)
{
    StepArgs a{};
    a.tab = c->ct1;
    a.cur = c->cur;
    a.R = c->R;
    a.block = c->cfg.block;
    a.tpa = c->cfg.tpa;
    a.M = c->cfg.M;
    a.n16 = c->cfg.n16;
    a.h = 0.5 * c->dt;
    a.c1 = c->c1;
    a.ushiftd = c->ushift;
    a.seed = c->seed;
    a.thermo = c->thermo;
    a.do_u = 1;
    a.do_svr = 0;
    a.svr_c = c->svr_c;
    return a;
}

// Rebuild lists and recompute forces + energies of replicas [r0, r0+nrep)
// at their current positions (a stopped boundary).
static int refresh_replicas(re_ctx* c, int r0, int nrep)
{
    const bool f64 = c->prec == RE_FP64;
    StepArgs a = base_args(c);
    a.force_all = 1;
    a.par = 0;
    for (int r = r0; r < r0 + nrep; ++r) {
        a.r0 = r;
        HIPCHK(c, launch_rebuild(f64, c->d, a, 1, c->N[r], c->wide_reorder, c->stream));
        a.tab = c->ctF;
        a.blk_off = c->cF_start[r];
        HIPCHK(c, launch_force(f64, kRefresh, c->d, a, c->cF_count[r], c->stream));
        HIPCHK(c, launch_energy(f64, c->d, a, 1, c->stream));
    }
    return 0;
}

static int check_overflow(re_ctx* c)
{
    uint32_t ov = 0;
    HIPCHK(c, hipMemcpyAsync(&ov, c->d.overflow, sizeof ov, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (ov) return fail(c, RE_EOVERFLOW, "a neighbour list exceeded its capacity of %d entries per atom", c->cfg.M);
    return 0;
}

// ---------------------------------------------------------------------------
// block tables
static void table_contiguous(const re_ctx* c, const std::vector<int>& apb, std::vector<int32_t>& brep,
                             std::vector<int32_t>& ba0, std::vector<int32_t>& start, std::vector<int32_t>& count)
{
    brep.clear();
    ba0.clear();
    start.assign(c->R, 0);
    count.assign(c->R, 0);
    for (int r = 0; r < c->R; ++r) {
        start[r] = (int)brep.size();
        for (int a0 = 0; a0 < c->N[r]; a0 += apb[r]) {
            brep.push_back(r);
            ba0.push_back(a0);
        }
        count[r] = (int)brep.size() - start[r];
    }
}

// XCD-aware table: consecutive block ids are dispatched round-robin over the
// 8 XCDs, so the blocks of one replica sit at ids of one residue mod 8 and
// share that XCD's L2; replicas are spread over the XCDs by atom count,
// largest first.
static void table_interleaved(const re_ctx* c, const std::vector<int>& apb, std::vector<int32_t>& brep,
                              std::vector<int32_t>& ba0)
{
    const int X = 8;
    std::vector<std::vector<std::pair<int, int>>> bins(X);
    std::vector<int64_t> load(X, 0);
    std::vector<int> order(c->R);
    for (int r = 0; r < c->R; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c->N[a] > c->N[b]; });
    for (int r : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (int a0 = 0; a0 < c->N[r]; a0 += apb[r]) bins[x].push_back({r, a0});
        load[x] += c->N[r];
    }
    size_t depth = 0;
    for (auto& b : bins) depth = std::max(depth, b.size());
    brep.clear();
    ba0.clear();
    for (size_t t = 0; t < depth; ++t)
        for (int x = 0; x < X; ++x) {
            const bool has = t < bins[x].size();
            brep.push_back(has ? bins[x][t].first : -1);
            ba0.push_back(has ? bins[x][t].second : 0);
        }
}

static int upload_table(re_ctx* c, const std::vector<int32_t>& brep, const std::vector<int32_t>& ba0, BlockTable& t)
{
    int rc;
    if ((rc = dalloc(c, &t.rep, brep.size())) || (rc = dalloc(c, &t.a0, ba0.size()))) return rc;
    HIPCHK(c, hipMemcpy(t.rep, brep.data(), brep.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(t.a0, ba0.data(), ba0.size() * 4, hipMemcpyHostToDevice));
    return 0;
}

static int build_tables(re_ctx* c)
{
    std::vector<int32_t> brep, ba0;
    int rc;
    // (the force kernels' blocks hold blockDim / tpa atoms of their replica)
    std::vector<int> apb1(c->R, c->cfg.block), apbF(c->R);
    for (int r = 0; r < c->R; ++r) apbF[r] = c->cfg.block / c->tpa_r[r];
    table_contiguous(c, apb1, brep, ba0, c->c1_start, c->c1_count);
    if ((rc = upload_table(c, brep, ba0, c->ct1))) return rc;
    table_contiguous(c, apbF, brep, ba0, c->cF_start, c->cF_count);
    if ((rc = upload_table(c, brep, ba0, c->ctF))) return rc;
    table_interleaved(c, apb1, brep, ba0);
    c->nbt1 = (int)brep.size();
    if ((rc = upload_table(c, brep, ba0, c->bt1))) return rc;
    table_interleaved(c, apbF, brep, ba0);
    c->nbtF = (int)brep.size();
    if ((rc = upload_table(c, brep, ba0, c->btF))) return rc;
    return 0;
}

// ---------------------------------------------------------------------------
// Lockstep engines.  A stopped boundary holds x_s, the full-step v_s and
// F_s = F(x_s).  From it, "start" runs B A O A of step s; the list is
// updated where the half-skin test fired; "force" evaluates F(x_{s+1}) and
// either stops (v_{s+1} = v + h F, F stored) or fuses the next step's first
// half (positions to the other buffer).  Stops happen at exchange steps, at
// the end of the call, and -- in the plain form -- after every step.
static int run_lockstep(re_ctx* c, int64_t n)
{
    const bool f64 = c->prec == RE_FP64;
    const bool plain = c->form == RE_PLAIN;
    const int R = c->R;
    StepArgs a = base_args(c);
    // the velocity rescale ends every step at a stopped boundary
    const bool svr = c->thermo == kThermoSVR;
    bool at_boundary = true;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t s = c->step;
        a.cur = c->cur;
        const bool xstep = ((s + 1) % c->Nx) == 0;
        const bool last = (i == n - 1);
        if (at_boundary) {
            a.step = s;
            a.apply_alpha = c->pending_alpha;
            if (plain) {
                a.tab = c->ct1;
                for (int r = 0; r < R; ++r) {
                    a.blk_off = c->c1_start[r];
                    HIPCHK(c, launch_start(f64, c->d, a, c->c1_count[r], c->stream));
                }
            } else {
                a.tab = c->bt1;
                a.blk_off = 0;
                HIPCHK(c, launch_start(f64, c->d, a, c->nbt1, c->stream));
            }
            c->pending_alpha = 0;
            a.apply_alpha = 0;
            at_boundary = false;
        }
        a.par = (int)((s + 1) & 1);
        a.force_all = 0;
        a.step = s + 1;
        const bool stop = plain || xstep || last || svr;
        const StepMode mode = !stop ? kFused : ((xstep || last) ? kStopEnergy : kStop);
        a.do_u = mode == kStopEnergy;
        a.do_svr = svr;
        const bool reduce = a.do_u || a.do_svr;
        if (plain) {
            for (int r = 0; r < R; ++r) {
                a.r0 = r;
                HIPCHK(c, launch_rebuild(f64, c->d, a, 1, c->N[r], c->wide_reorder, c->stream));
                a.tab = c->ctF;
                a.blk_off = c->cF_start[r];
                HIPCHK(c, launch_force(f64, mode, c->d, a, c->cF_count[r], c->stream));
                if (reduce) HIPCHK(c, launch_energy(f64, c->d, a, 1, c->stream));
            }
        } else {
            a.r0 = 0;
            HIPCHK(c, launch_rebuild(f64, c->d, a, R, c->total_atoms, c->wide_reorder, c->stream));
            a.blk_off = 0;
            a.tab = c->btF;
            const bool timed = c->prof && mode == kFused && c->ev_used + 2 <= (int)c->ev.size();
            if (timed) HIPCHK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
            HIPCHK(c, launch_force(f64, mode, c->d, a, c->nbtF, c->stream));
            if (timed) {
                HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
                c->ev_used += 2;
            }
            if (reduce) HIPCHK(c, launch_energy(f64, c->d, a, R, c->stream));
        }
        if (stop) {
            at_boundary = true;
            if (svr) c->pending_alpha = 1;
            if (xstep) {
                HIPCHK(c, launch_exchange(c->d, R, c->next_attempt, c->seed, c->c1 * c->c1, -1, c->cfg.log_cap,
                                          s + 1, c->xmaxd, c->stream));
                c->next_attempt += 1;
                c->pending_alpha = 1;
            }
        } else {
            c->cur ^= 1;
        }
        c->step = s + 1;
    }
    if (n > 0) HIPCHK(c, launch_set_steps(c->d, R, c->step, c->stream));
    return check_overflow(c);
}

template <class T>
static int d2h(re_ctx* c, T* dst, const T* src, size_t n)
{
    HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
}

// ---------------------------------------------------------------------------
// Persistent engine: team planning.  One 1024-thread workgroup per CU can be
// resident (the reorder's cell counts fill most of the LDS), so at most
// #CUs workgroups run; block ids of one residue mod 8 go to the same XCD.
// Replica r gets a team of t_r workgroups (at least one, at most one per
// 256 atoms) in proportion to its weight w_r: its atoms, or its atoms times
// the cost of its measured step (list updates included) when the teams are
// rebalanced.  With at least 8 replicas every team stays on one XCD, so
// that a replica's data stays in one L2 and its barrier needs no L2
// write-back: the replicas are dealt to the XCDs largest weight first,
// each to the XCD with the least weight so far (at most ceil(R/8) each),
// and each XCD's CUs are split among its replicas by weight.  With fewer
// replicas (or an explicit team size) the teams are sized over the whole
// device and placed largest first, on one XCD where they fit.
static int plan_persistent(re_ctx* c, int team_opt, const std::vector<double>* weight = nullptr)
{
    int dev = 0, cus = 0, occ = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(c, persist_occupancy(c->prec == RE_FP64, c->cfg.n16 != 0, c->cfg.tpa, c->thermo == kThermoSVR, &occ));
    const int cap = cus * std::max(0, occ);
    const int R = c->R;
    c->pers_ok = false;
    if (cap < R) {
        c->pers_why = "the persistent engine needs one resident workgroup per replica (" + std::to_string(cap) +
                      " available, " + std::to_string(R) + " replicas)";
        return 0;
    }
    std::vector<double> w(R);
    for (int r = 0; r < R; ++r) w[r] = weight ? (*weight)[r] : (double)c->N[r];
    const int X = 8, per = (cap + X - 1) / X;
    auto tcap = [&](int r) { return std::max(1, (c->N[r] + 255) / 256); };
    std::vector<int32_t> brep(X * per, -1), bmem(X * per, 0), bsize(X * per, 1), bid(X * per, 0);
    std::vector<int> t(R, 1);
    if (team_opt <= 0 && R >= X && cap % X == 0) {
        // deal the replicas to the XCDs, then split each XCD's CUs
        std::vector<int> order(R), xof(R);
        for (int r = 0; r < R; ++r) order[r] = r;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
        const int maxper = (R + X - 1) / X;
        std::vector<double> wx(X, 0.0);
        std::vector<std::vector<int>> members(X);
        for (int r : order) {
            int best = -1;
            for (int x = 0; x < X; ++x)
                if ((int)members[x].size() < maxper && (best < 0 || wx[x] < wx[best])) best = x;
            members[best].push_back(r);
            wx[best] += w[r];
            xof[r] = best;
        }
        for (int x = 0; x < X; ++x) {
            auto& m = members[x];
            if (m.empty()) continue;
            int used = 0;
            for (int r : m) {
                t[r] = std::max(1, std::min(tcap(r), (int)std::floor(per * w[r] / wx[x])));
                used += t[r];
            }
            // the XCD's remaining CUs, one at a time, to the heaviest replica
            // per workgroup that can still grow
            while (used < per) {
                int pick = -1;
                for (int r : m)
                    if (t[r] < tcap(r) && (pick < 0 || w[r] / t[r] > w[pick] / t[pick])) pick = r;
                if (pick < 0) break;
                t[pick] += 1;
                used += 1;
            }
            while (used > per) {  // (only when there are more replicas than CUs here)
                int pick = -1;
                for (int r : m)
                    if (t[r] > 1 && (pick < 0 || w[r] / t[r] < w[pick] / t[pick])) pick = r;
                if (pick < 0) break;
                t[pick] -= 1;
                used -= 1;
            }
            int k = 0;
            for (int r : m)
                for (int mm = 0; mm < t[r]; ++mm, ++k) {
                    const int b = x + X * k;
                    brep[b] = r;
                    bmem[b] = mm;
                    bsize[b] = t[r];
                    bid[b] = r;
                }
            if (k > per) {
                c->pers_why = "team placement exceeds the resident workgroups of an XCD";
                return 0;
            }
        }
    } else {
        if (team_opt > 0) {
            for (int r = 0; r < R; ++r) t[r] = team_opt;
        } else {
            double tot = 0;
            for (int r = 0; r < R; ++r) tot += w[r];
            for (int r = 0; r < R; ++r) t[r] = std::max(1, (int)std::floor(cap * w[r] / tot));
        }
        for (int r = 0; r < R; ++r) t[r] = std::max(1, std::min(t[r], tcap(r)));
        for (;;) {
            int sum = 0, big = 0;
            for (int r = 0; r < R; ++r) {
                sum += t[r];
                if (t[r] > t[big]) big = r;
            }
            if (sum <= cap) break;
            t[big] -= 1;
        }
        // place teams: largest first, onto the XCD with the most free slots
        std::vector<int> freec(X, per), order(R);
        for (int r = 0; r < R; ++r) order[r] = r;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return t[a] > t[b]; });
        std::vector<int> used(X, 0);
        for (int k = 0; k < R; ++k) {
            const int r = order[k];
            int x = (int)(std::max_element(freec.begin(), freec.end()) - freec.begin());
            for (int m = 0; m < t[r]; ++m) {
                if (freec[x] == 0) x = (int)(std::max_element(freec.begin(), freec.end()) - freec.begin());
                const int b = x + X * used[x];
                used[x] += 1;
                freec[x] -= 1;
                brep[b] = r;
                bmem[b] = m;
                bsize[b] = t[r];
                bid[b] = r;
            }
        }
    }
    int nblk = 0;
    for (int b = 0; b < X * per; ++b)
        if (brep[b] >= 0) nblk = b + 1;
    if (nblk > cap) {
        c->pers_why = "team placement exceeds the resident workgroups";
        return 0;
    }
    int rc;
    if (!c->t_rep) {
        if ((rc = dalloc(c, &c->t_rep, X * per)) || (rc = dalloc(c, &c->t_mem, X * per)) ||
            (rc = dalloc(c, &c->t_size, X * per)) || (rc = dalloc(c, &c->t_id, X * per)) ||
            (rc = dalloc(c, &c->bar, 64 * (size_t)R)))
            return rc;
    }
    HIPCHK(c, hipMemcpy(c->t_rep, brep.data(), brep.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->t_mem, bmem.data(), bmem.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->t_size, bsize.data(), bsize.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->t_id, bid.data(), bid.size() * 4, hipMemcpyHostToDevice));
    c->pnblk = nblk;
    c->pnteams = R;
    c->team_of = t;
    c->pers_ok = true;
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        (void)hipGraphDestroy(c->graph);
        c->gexec = nullptr;
        c->graph = nullptr;
    }
    return 0;
}

// Rebalancing of the teams from the measured list-update rates (persistent
// engine, automatic team sizes): once every replica has done kBalanceSteps
// steps since the last plan, replica r is weighted by N_r (1 + kListCost u_r),
// u_r its list updates per step in that window and kListCost the cost of
// one update (reorder, list build and their barriers) in units of one
// step's force phase, about 4 at 4000 atoms per replica.  The teams are
// re-planned (and the launch graph re-captured) when a team changes size.
// Hot replicas update their lists about twice as often as cold ones, so
// with equal teams the cold ones wait for them at every synchronous
// exchange.  Results do not depend on the teams.
constexpr int64_t kBalanceSteps = 500;
constexpr double kListCost = 4.0;

static int maybe_rebalance(re_ctx* c, const int64_t* steps)
{
    const int R = c->R;
    if (!c->balance || c->team_opt > 0 || c->plan_steps.empty()) return 0;
    int64_t dmin = INT64_MAX;
    for (int r = 0; r < R; ++r) dmin = std::min(dmin, steps[r] - c->plan_steps[r]);
    if (dmin < kBalanceSteps) return 0;
    std::vector<int64_t> reb(R);
    int rc = d2h(c, reb.data(), c->d.rebuilds, R);
    if (rc) return rc;
    std::vector<double> w(R);
    for (int r = 0; r < R; ++r) {
        const double u = (double)(reb[r] - c->plan_reb[r]) / (double)std::max<int64_t>(1, steps[r] - c->plan_steps[r]);
        w[r] = (double)c->N[r] * (1.0 + kListCost * u);
    }
    c->plan_steps.assign(steps, steps + R);
    c->plan_reb = reb;
    const std::vector<int> before = c->team_of;
    if ((rc = plan_persistent(c, 0, &w))) return rc;
    if (!c->pers_ok) {  // (cannot happen for a plan that fitted before; keep the old one)
        return plan_persistent(c, 0, nullptr);
    }
    c->rebalanced += c->team_of != before ? 1 : 0;
    return 0;
}

static PersistArgs persist_args(re_ctx* c)
{
    PersistArgs pa{};
    pa.sa = base_args(c);
    pa.st = c->ps;
    pa.call = c->d_call;
    pa.team_rep = c->t_rep;
    pa.team_mem = c->t_mem;
    pa.team_size = c->t_size;
    pa.team_id = c->t_id;
    pa.bar = c->bar;
    pa.Nx = c->Nx;
    pa.c1sq = c->c1 * c->c1;
    pa.log_cap = c->cfg.log_cap;
    pa.timeout = (uint64_t)(c->watchdog * 1e8);
    pa.bar_mode = c->bar_mode;
    pa.xmaxd = c->xmaxd;
    pa.delay_ticks = (uint32_t)c->delay_us * 100u;
    return pa;
}

// One persistent launch (captured once into a HIP graph of the per-call
// reset kernel and the persistent kernel, replayed for every call; the
// per-call parameters live in device memory and are copied before).
static int run_persistent(re_ctx* c, int64_t n)
{
    if (!c->pers_ok) return fail(c, RE_ESTATE, "%s", c->pers_why.c_str());
    const int R = c->R;
    int rc;
    // teams rebalanced from the list-update rates measured so far (the step
    // counts are those the previous call read back)
    {
        const int64_t* st = reinterpret_cast<const int64_t*>(c->h_stat + 8) + R;
        if (c->stat_valid && (rc = maybe_rebalance(c, st))) return rc;
        if (!c->pers_ok) return fail(c, RE_ESTATE, "%s", c->pers_why.c_str());
    }
    // per-call parameters through pinned memory: the copy is queued and the
    // host goes on; every call ends with a synchronisation, so the staging
    // buffer is free again when the next call writes it
    CallParams& cp = *c->h_call;
    cp = CallParams{};
    cp.cur0 = c->cur;
    cp.k0 = c->next_attempt;
    cp.sched = c->d_sched;
    cp.apply_alpha = c->pending_alpha;
    if (!c->sched.empty()) {
        cp.mode = kModeSchedule;
        cp.A = c->sched_A;
        if (c->sched_cap < (int64_t)c->sched.size()) {
            if ((rc = dalloc(c, &c->d_sched, c->sched.size()))) return rc;
            c->sched_cap = (int64_t)c->sched.size();
            cp.sched = c->d_sched;
        }
        HIPCHK(c, hipMemcpyAsync(c->d_sched, c->sched.data(), c->sched.size() * 8, hipMemcpyHostToDevice, c->stream));
    } else {
        cp.mode = c->xmode == RE_ASYNC ? kModeAsync : kModeSync;
        cp.n = n;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_call, c->h_call, sizeof(CallParams), hipMemcpyHostToDevice, c->stream));
    c->pending_alpha = 0;
    const bool f64 = c->prec == RE_FP64;
    if (!c->gexec) {
        const PersistArgs pa = persist_args(c);
        hipStream_t cs;
        HIPCHK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) e = launch_persist(f64, c->d, pa, c->pnblk, c->pnteams, cs);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            c->gexec = nullptr;
            return fail(c, RE_EDEVICE, "capturing the persistent launch: %s", hipGetErrorString(e));
        }
        c->graph = g;
    }
    const bool timed = c->prof && c->ev_used + 2 <= (int)c->ev.size();
    if (timed) HIPCHK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    if (timed) {
        HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
        c->ev_used += 2;
    }
    // error bits, overflow flag, next attempts and step counts: one copy, one
    // synchronisation
    HIPCHK(c, hipMemcpyAsync(c->h_stat, c->d_stat, 8 + 16 * (size_t)R, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint32_t err = 0, ov = 0;
    std::memcpy(&err, c->h_stat, 4);
    std::memcpy(&ov, c->h_stat + 4, 4);
    const int64_t* katt = reinterpret_cast<const int64_t*>(c->h_stat + 8);
    const int64_t* steps = katt + R;
    c->next_attempt = *std::max_element(katt, katt + R);
    c->step = steps[0];
    c->stat_valid = true;
    c->sched.clear();
    c->sched_A = 0;
    if (err & kErrTimeout)
        return fail(c, RE_ETIMEOUT, "a device-side wait made no progress for %.1f s; the run was aborted", c->watchdog);
    if (ov) return fail(c, RE_EOVERFLOW, "a neighbour list exceeded its capacity of %d entries per atom", c->cfg.M);
    return 0;
}

// ---------------------------------------------------------------------------
// C ABI
extern "C" {

int re_create(re_ctx** out, int R, const int32_t* N_atoms, const double* T_ladder, double rho, double r_c,
              double skin, double dt, int N_x, uint64_t seed, const re_options* opt)
{
    if (!out) return fail(nullptr, RE_EINVAL, "out is NULL");
    *out = nullptr;
    re_options o{};
    if (opt) o = *opt;
    if (R < 1 || R > 4096) return fail(nullptr, RE_EINVAL, "R must be in [1, 4096], got %d", R);
    if (!N_atoms || !T_ladder) return fail(nullptr, RE_EINVAL, "N_atoms and T_ladder must not be NULL");
    if (!(r_c > 0) || !(skin >= 0) || !(dt > 0) || N_x < 1)
        return fail(nullptr, RE_EINVAL, "need r_c > 0, skin >= 0, dt > 0, N_x >= 1");
    if (!o.rho_per_replica && !(rho > 0)) return fail(nullptr, RE_EINVAL, "rho must be > 0");
    for (int r = 0; r < R; ++r) {
        if (N_atoms[r] < 2) return fail(nullptr, RE_EINVAL, "N_atoms[%d] = %d < 2", r, N_atoms[r]);
        if (N_atoms[r] > (1 << 26)) return fail(nullptr, RE_EINVAL, "N_atoms[%d] too large", r);
        if (!(T_ladder[r] > 0)) return fail(nullptr, RE_EINVAL, "T_ladder[%d] must be > 0", r);
        if (r && !(T_ladder[r] > T_ladder[r - 1]))
            return fail(nullptr, RE_EINVAL, "T_ladder must be strictly ascending");
        if (o.rho_per_replica && !(o.rho_per_replica[r] > 0))
            return fail(nullptr, RE_EINVAL, "rho_per_replica[%d] must be > 0", r);
    }
    if (o.precision != RE_MIXED && o.precision != RE_FP64) return fail(nullptr, RE_EINVAL, "bad precision");
    if (o.form != RE_BATCHED && o.form != RE_PLAIN) return fail(nullptr, RE_EINVAL, "bad form");
    if (o.batched_engine != RE_LOCKSTEP && o.batched_engine != RE_PERSISTENT)
        return fail(nullptr, RE_EINVAL, "bad batched_engine");
    if (o.exchange_mode != RE_SYNC && o.exchange_mode != RE_ASYNC) return fail(nullptr, RE_EINVAL, "bad exchange_mode");
    if (o.team_barrier != RE_BARRIER_AUTO && o.team_barrier != RE_BARRIER_AGENT)
        return fail(nullptr, RE_EINVAL, "bad team_barrier");
    if (o.exchange_max_distance < 0) return fail(nullptr, RE_EINVAL, "exchange_max_distance must be >= 0");
    if (o.debug_delay_us < 0 || o.debug_delay_us > 100000)
        return fail(nullptr, RE_EINVAL, "debug_delay_us must be in [0, 100000]");
    if (o.threads_per_atom && o.threads_per_atom != 1 && o.threads_per_atom != 2 && o.threads_per_atom != 4 &&
        o.threads_per_atom != 8)
        return fail(nullptr, RE_EINVAL, "threads_per_atom must be 1, 2, 4 or 8");
    if (o.threads_per_atom_per_replica)
        for (int r = 0; r < R; ++r) {
            const int t = o.threads_per_atom_per_replica[r];
            if (t != 1 && t != 2 && t != 4 && t != 8)
                return fail(nullptr, RE_EINVAL, "threads_per_atom_per_replica[%d] must be 1, 2, 4 or 8", r);
        }
    if (o.block_size && o.block_size != 64 && o.block_size != 128 && o.block_size != 256)
        return fail(nullptr, RE_EINVAL, "block_size must be 64, 128 or 256");
    const double gamma = o.gamma_set ? o.gamma : 1.0;
    if (!(gamma >= 0)) return fail(nullptr, RE_EINVAL, "gamma must be >= 0");
    if (o.thermostat != RE_LANGEVIN && o.thermostat != RE_SVR) return fail(nullptr, RE_EINVAL, "bad thermostat");
    if (!(o.svr_tau >= 0)) return fail(nullptr, RE_EINVAL, "svr_tau must be >= 0");
    const double tau = o.svr_tau > 0 ? o.svr_tau : 0.5;
    std::vector<int32_t> tuned_tpa;  // per replica, from the autotuner's size classes
    if (o.autotune && o.form == RE_BATCHED) {
        // the engine and lanes per atom of this size class: cached, or timed
        const std::string key =
            tune_key(R, N_atoms, o.rho_per_replica, rho, r_c, skin, o.precision, o.exchange_mode, o.thermostat);
        TuneChoice ch{};
        if (!tune_lookup(o.tune_cache, key, ch)) {
            const int rt = tune_run(R, N_atoms, T_ladder, rho, r_c, skin, dt, N_x, seed, o, ch);
            if (rt != RE_OK) return fail(nullptr, rt, "autotuning failed: %s", g_noctx_error.c_str());
            tune_store(o.tune_cache, key, ch);
        }
        o.batched_engine = ch.engine;
        o.threads_per_atom = ch.tpa;
        if (ch.block) o.block_size = ch.block;
        o.autotune = 0;
        tuned_tpa.assign(R, ch.tpa);
        bool per_class = false;
        for (int r = 0; r < R; ++r) {
            const int k = tune_class(N_atoms[r]);
            if (ch.cls_tpa[k]) tuned_tpa[r] = ch.cls_tpa[k];
            per_class |= tuned_tpa[r] != ch.tpa;
        }
        o.threads_per_atom_per_replica = per_class ? tuned_tpa.data() : nullptr;
    }
    if (o.form == RE_PLAIN && o.exchange_mode == RE_ASYNC)
        return fail(nullptr, RE_EINVAL, "the plain per-replica form runs synchronous exchanges only");
    const double rlist = r_c + skin;
    std::vector<double> rho_r(R), L_r(R);
    for (int r = 0; r < R; ++r) {
        rho_r[r] = o.rho_per_replica ? o.rho_per_replica[r] : rho;
        L_r[r] = box_side(N_atoms[r], rho_r[r]);
        if (!(rlist < 0.5 * L_r[r]))
            return fail(nullptr, RE_EINVAL, "r_c + skin = %g must be < L/2 = %g (replica %d)", rlist, 0.5 * L_r[r], r);
    }

    re_ctx* c = new re_ctx();
    c->R = R;
    c->prec = o.precision;
    c->form = o.form;
    c->engine = o.batched_engine;
    c->xmode = o.exchange_mode;
    c->rc = r_c;
    c->skin = skin;
    c->dt = dt;
    c->gamma = gamma;
    c->Nx = N_x;
    c->seed = seed;
    c->watchdog = o.watchdog_seconds > 0 ? o.watchdog_seconds : 10.0;
    c->bar_mode = o.team_barrier == RE_BARRIER_AGENT ? 0 : 1;
    c->N.assign(N_atoms, N_atoms + R);
    c->Tl.assign(T_ladder, T_ladder + R);
    c->rho = rho_r;
    c->L = L_r;
    {
        const double ir6 = 1.0 / (r_c * r_c * r_c * r_c * r_c * r_c);
        c->ushift = 4.0 * (ir6 * ir6 - ir6);
    }
    c->thermo = o.thermostat == RE_SVR ? kThermoSVR : kThermoLangevin;
    c->xmaxd = o.exchange_max_distance > 0 ? o.exchange_max_distance : 1;
    c->delay_us = o.debug_delay_us;
    // under the velocity rescale the integrator has no friction and no noise
    c->c1 = c->thermo == kThermoSVR ? 1.0 : std::exp(-c->gamma * dt);
    c->svr_c = std::exp(-dt / tau);

    // launch configuration
    c->cfg.block = o.block_size ? o.block_size : 256;
    c->cfg.tpa = o.threads_per_atom ? o.threads_per_atom : 4;
    c->tpa_r.assign(R, c->cfg.tpa);
    if (o.threads_per_atom_per_replica) {
        // lanes per atom per replica; the kernels dispatch per replica
        // (cfg.tpa = 0) unless every replica has the same
        for (int r = 0; r < R; ++r) c->tpa_r[r] = o.threads_per_atom_per_replica[r];
        const bool uniform = std::all_of(c->tpa_r.begin(), c->tpa_r.end(), [&](int t) { return t == c->tpa_r[0]; });
        c->cfg.tpa = uniform ? c->tpa_r[0] : 0;
    }
    c->cfg.log_cap = o.log_capacity > 0 ? o.log_capacity : (int64_t)1 << 18;
    double rho_max = 0;
    for (double q : c->rho) rho_max = std::max(rho_max, q);
    {
        // expected neighbours within the list radius, with room for density
        // fluctuations; a multiple of 32 (whole groups of 4 rows at every
        // threads_per_atom)
        const double expect = 4.18879020478639 * rlist * rlist * rlist * rho_max;
        c->cfg.M = ((int)std::ceil(1.4 * expect) + 32 + 31) / 32 * 32;
    }

    // 16-bit list entries (the neighbour's slot) when every replica of the
    // mixed form has at most 65536 atoms; 32-bit byte offsets otherwise
    c->cfg.n16 = c->prec == RE_MIXED && *std::max_element(N_atoms, N_atoms + R) <= 65536 ? 1 : 0;
    const int64_t esz = c->cfg.n16 ? 2 : 4;

    // per-replica layout
    c->rep.resize(R);
    int64_t slots = 0, nl = 0;
    int cells = 0;
    for (int r = 0; r < R; ++r) {
        RepDev& rd = c->rep[r];
        std::memset(&rd, 0, sizeof rd);
        rd.N = c->N[r];
        rd.Np = (rd.N + 63) / 64 * 64;
        rd.tpa = c->tpa_r[r];
        rd.base = (int32_t)slots;
        slots += rd.Np;
        rd.L = c->L[r];
        c->nmax = std::max(c->nmax, rd.N);
        c->total_atoms += rd.N;
        // fine cells: side >= r_list / 2 (the list build scans 5 x 5 x 5 cells)
        int nc = (int)std::floor(rd.L / (0.5 * rlist * (1.0 + 1e-5)));
        nc = std::max(1, std::min(nc, kMaxCellsPerSide));
        rd.ncell = nc;
        {
            const double q = rlist * (1.0 + 1e-4) * nc / rd.L;
            rd.rlcell2 = (float)(q * q);
        }
        rd.cell_base = cells;
        cells += nc * nc * nc + 1;
        c->cells_max = std::max(c->cells_max, nc * nc * nc);
        rd.nl_base = nl;
        nl += (int64_t)rd.Np * c->cfg.M;
        // list entries of one replica are addressed with 32-bit byte offsets
        // (with the slack rows read past the block)
        const int64_t nl_bytes = ((int64_t)rd.Np * c->cfg.M + (int64_t)kListSlackRows * 8 * rd.Np) * esz;
        if (nl_bytes >= ((int64_t)1 << 32)) {
            delete c;
            return fail(nullptr, RE_EINVAL, "replica %d: its neighbour-list block (%lld bytes) reaches 2^32 bytes", r,
                        (long long)nl_bytes);
        }
        if (c->prec == RE_MIXED) {
            rd.s = rd.L * 0x1p-32;
            rd.inv_s = 0x1p32 / rd.L;
        } else {
            rd.s = 1.0;
            rd.inv_s = 1.0;
        }
        rd.sf = (float)rd.s;
        rd.inv_sf = (float)rd.inv_s;
        rd.inv_s2f = (float)(rd.inv_s * rd.inv_s);
        const double rcu = r_c * rd.inv_s, limu = 0.5 * skin * rd.inv_s;
        rd.rc2f = (float)(rcu * rcu);
        rd.near_lo = (float)(rcu * rcu * (1.0 - 0x1p-20));
        rd.near_hi = (float)(rcu * rcu * (1.0 + 0x1p-20));
        rd.lim2f = (float)(limu * limu);
        // mixed list build: coordinates truncated to the top 16 bits differ
        // from the true ones by less than one step of L 2^-16 each, so a pair
        // closer than r_list has a key difference shorter than r_list / step
        // + sqrt 3.  The radius carries a 2e-6 relative margin, so that FP32
        // rounding in the half-skin test can never let a pair unlisted at the
        // update come within r_c before the next update.
        {
            const double rq = rlist * (1.0 + 2e-6) * 0x1p16 / rd.L + 1.7320508075688772 + 1e-9;
            rd.rl2q = (uint32_t)std::min(std::ceil(rq * rq), 4294967295.0);
        }
        rd.rc2d = r_c * r_c;
        rd.rl2d = rlist * rlist * (1.0 + 1e-12);
        rd.lim2d = 0.25 * skin * skin;
        if (c->prec == RE_MIXED) {
            const long double q = (long double)r_c * (long double)0x1p32 / (long double)rd.L;
            rd.rc2_exact = (uint64_t)ceill(q * q);
        }
    }
    c->total_slots = slots;
    // one workgroup reorders a replica of a few thousand atoms in tens of
    // microseconds; larger replicas are reordered by grid-wide passes
    c->wide_reorder = c->nmax >= 16384;
    c->total_cells = cells;

    int rc = 0;
    auto bail = [&](int code) {
        std::string m = c->err;
        re_destroy(c);
        return fail(nullptr, code, "%s", m.c_str());
    };
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, RE_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        c->own_stream = true;
    }
    DevState& d = c->d;
#define ALLOC(p, n) \
    if ((rc = dalloc(c, &(p), (n))) != 0) return bail(rc);
    if (c->prec == RE_MIXED) {
        ALLOC(d.posi[0], slots + kPosSlack);
        ALLOC(d.posi[1], slots + kPosSlack);
        ALLOC(d.velf, slots);
        ALLOC(d.frcf, slots);
        ALLOC(d.xrefi, slots);
        ALLOC(d.epotf, slots);
        ALLOC(d.veltf, slots);
    } else {
        ALLOC(d.posd[0], slots + kPosSlack);
        ALLOC(d.posd[1], slots + kPosSlack);
        ALLOC(d.veld, slots);
        ALLOC(d.frcd, slots);
        ALLOC(d.xrefd, slots);
        ALLOC(d.epotd, slots);
        ALLOC(d.veltd, slots);
    }
    ALLOC(d.perm, slots);
    ALLOC(d.cellid, slots);
    ALLOC(d.rank, slots);
    ALLOC(d.cell_start, cells);
    {
        unsigned char* nlp = nullptr;
        const size_t nl_bytes_all = (size_t)((nl + (int64_t)kListSlackRows * 8 * ((c->nmax + 63) / 64 * 64)) * esz);
        ALLOC(nlp, nl_bytes_all);
        d.nl = nlp;
        // zeroed: every entry of a replica's block then names one of its
        // atoms (slot 0) until a list build writes it, so the force loops'
        // reads past an atom's rows stay inside the replica
        if (hipMemset(nlp, 0, nl_bytes_all) != hipSuccess) {
            c->err = "hipMemset of the neighbour lists failed";
            return bail(RE_EDEVICE);
        }
    }
    ALLOC(d.nn, slots);
    ALLOC(d.rep, R);
    ALLOC(d.slot, R);
    ALLOC(d.Tl, R);
    ALLOC(d.c2, R);
    ALLOC(d.alpha, R);
    ALLOC(d.U, R);
    ALLOC(d.flag, 2 * R);
    ALLOC(d.rebuilds, R);
    ALLOC(d.attempts, R);
    ALLOC(d.accepts, R);
    ALLOC(d.log, c->cfg.log_cap);
    ALLOC(d.log_count, 1);
    // the status block: error bits, overflow flag, next attempts, step counts
    ALLOC(c->d_stat, 8 + 16 * (size_t)R);
    c->ps.err = reinterpret_cast<uint32_t*>(c->d_stat);
    d.overflow = reinterpret_cast<uint32_t*>(c->d_stat + 4);
    c->ps.katt = reinterpret_cast<int64_t*>(c->d_stat + 8);
    d.steps = c->ps.katt + R;
    ALLOC(d.fq, 4 * slots);
    ALLOC(d.wtab, 4 * (size_t)R + 4);
    if (c->thermo == kThermoSVR) ALLOC(d.svrq, slots);
    ALLOC(c->ps.slotbuf, 2 * R);
    ALLOC(c->ps.post, R);
    ALLOC(c->ps.upost, 2 * R);
    ALLOC(c->ps.spost, 2 * R);
    ALLOC(c->ps.apend, R);
    ALLOC(c->ps.jprev, R);
    ALLOC(c->ps.ctl, 2 * R);
    ALLOC(c->ps.xdone, 1);
    ALLOC(c->ps.trig, 1);
    ALLOC(c->ps.parked, 1);
    ALLOC(c->ps.reach, 1);
    ALLOC(c->ps.beat, 1);
    ALLOC(c->ps.abort, 1);
    ALLOC(c->ps.xmask, R);
    ALLOC(c->d_call, 1);
#undef ALLOC
    {
        void* h1 = nullptr;
        void* h2 = nullptr;
        if (hipHostMalloc(&h1, sizeof(CallParams), hipHostMallocDefault) != hipSuccess ||
            (c->pinned.push_back(h1), hipHostMalloc(&h2, 8 + 16 * (size_t)R, hipHostMallocDefault) != hipSuccess)) {
            c->err = "hipHostMalloc of the call staging failed";
            return bail(RE_ENOMEM);
        }
        c->pinned.push_back(h2);
        c->h_call = static_cast<CallParams*>(h1);
        c->h_stat = static_cast<unsigned char*>(h2);
    }
    if ((rc = build_tables(c))) return bail(rc);

    // per-replica constants and bookkeeping
    std::vector<int32_t> slot(R);
    std::vector<double> c2(R), one(R, 1.0), zero(R, 0.0);
    for (int r = 0; r < R; ++r) {
        slot[r] = r;
        c2[r] = std::sqrt((1.0 - c->c1 * c->c1) * c->Tl[r]);
    }
    std::vector<int64_t> z64(R, 0);
    std::vector<uint32_t> z32(2 * R, 0);
    std::vector<int32_t> zs(slots, 0);
    hipError_t e = hipSuccess;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    cp(d.rep, c->rep.data(), R * sizeof(RepDev));
    cp(d.slot, slot.data(), R * 4);
    cp(d.Tl, c->Tl.data(), R * 8);
    cp(d.c2, c2.data(), R * 8);
    cp(d.alpha, one.data(), R * 8);
    cp(d.U, zero.data(), R * 8);
    cp(d.rebuilds, z64.data(), R * 8);
    cp(d.steps, z64.data(), R * 8);
    cp(d.attempts, z64.data(), R * 8);
    cp(d.accepts, z64.data(), R * 8);
    cp(d.log_count, z64.data(), 8);
    cp(d.overflow, z32.data(), 4);
    cp(d.flag, z32.data(), 2 * R * 4);
    cp(d.nn, zs.data(), slots * 4);
    cp(c->ps.post, z64.data(), R * 8);
    cp(c->ps.apend, z32.data(), R * 4);
    cp(c->ps.katt, z64.data(), R * 8);
    cp(c->ps.jprev, z64.data(), R * 8);
    cp(c->ps.err, z32.data(), 4);
    if (e != hipSuccess) {
        c->err = std::string("initial copies failed: ") + hipGetErrorString(e);
        return bail(RE_EDEVICE);
    }

    // initial state, built on host threads in parallel over replicas
    {
        std::vector<std::vector<double>> xs(R), vs(R);
        const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nth; ++t)
            th.emplace_back([&, t]() {
                for (int r = (int)t; r < R; r += (int)nth) init_replica(c->N[r], c->L[r], c->Tl[r], seed, r, xs[r], vs[r]);
            });
        for (auto& t : th) t.join();
        for (int r = 0; r < R; ++r) {
            if ((rc = upload_replica(c, r, xs[r].data(), vs[r].data()))) return bail(rc);
            std::vector<double>().swap(xs[r]);
            std::vector<double>().swap(vs[r]);
        }
    }
    if ((rc = refresh_replicas(c, 0, R)) || (rc = check_overflow(c))) return bail(rc);
    c->team_opt = o.team_size;
    c->balance = o.team_balance != 0;
    if (c->form == RE_BATCHED && (rc = plan_persistent(c, o.team_size))) return bail(rc);
    if (c->form == RE_BATCHED && c->pers_ok) {
        // the first window of the team rebalancing starts here
        std::memset(c->h_stat, 0, 8 + 16 * (size_t)R);
        c->stat_valid = true;
        c->plan_steps.assign(R, 0);
        c->plan_reb.assign(R, 0);
        if ((rc = d2h(c, c->plan_reb.data(), c->d.rebuilds, R))) return bail(rc);
    }
    if (c->xmode == RE_ASYNC && !c->pers_ok) {
        c->err = "asynchronous exchange needs the persistent engine: " + c->pers_why;
        return bail(RE_EINVAL);
    }
    *out = c;
    return RE_OK;
}

int re_step(re_ctx* c, int64_t n)
{
    if (!c) return fail(nullptr, RE_EINVAL, "ctx is NULL");
    if (n < 0) return fail(c, RE_EINVAL, "n must be >= 0");
    if (n == 0 && c->sched.empty()) return RE_OK;
    if (c->xmode == RE_ASYNC || (c->form == RE_BATCHED && c->engine == RE_PERSISTENT)) return run_persistent(c, n);
    return run_lockstep(c, n);
}

int re_exchange(re_ctx* c)
{
    if (!c) return fail(nullptr, RE_EINVAL, "ctx is NULL");
    HIPCHK(c, launch_exchange(c->d, c->R, c->next_attempt, c->seed, c->c1 * c->c1, -1, c->cfg.log_cap, c->step,
                              c->xmaxd, c->stream));
    c->next_attempt += 1;
    c->pending_alpha = 1;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RE_OK;
}

int re_query_energies(re_ctx* c, double* U)
{
    if (!c || !U) return fail(c, RE_EINVAL, "NULL argument");
    return d2h(c, U, c->d.U, c->R);
}

int re_query_slots(re_ctx* c, int32_t* slot)
{
    if (!c || !slot) return fail(c, RE_EINVAL, "NULL argument");
    return d2h(c, slot, c->d.slot, c->R);
}

int re_query_temps(re_ctx* c, double* T)
{
    if (!c || !T) return fail(c, RE_EINVAL, "NULL argument");
    std::vector<int32_t> s(c->R);
    int rc = d2h(c, s.data(), c->d.slot, c->R);
    if (rc) return rc;
    for (int r = 0; r < c->R; ++r) T[r] = c->Tl[s[r]];
    return RE_OK;
}

int re_query_acceptance(re_ctx* c, int64_t* att, int64_t* acc)
{
    if (!c) return fail(nullptr, RE_EINVAL, "ctx is NULL");
    const int n = c->R - 1;
    if (n <= 0) return RE_OK;
    int rc;
    if (att && (rc = d2h(c, att, c->d.attempts, n))) return rc;
    if (acc && (rc = d2h(c, acc, c->d.accepts, n))) return rc;
    return RE_OK;
}

int re_query_steps(re_ctx* c, int64_t* steps, int64_t* rebuilds)
{
    if (!c) return fail(nullptr, RE_EINVAL, "ctx is NULL");
    int rc;
    if (steps && (rc = d2h(c, steps, c->d.steps, c->R))) return rc;
    if (rebuilds && (rc = d2h(c, rebuilds, c->d.rebuilds, c->R))) return rc;
    return RE_OK;
}

int re_query_box(re_ctx* c, double* L)
{
    if (!c || !L) return fail(c, RE_EINVAL, "NULL argument");
    for (int r = 0; r < c->R; ++r) L[r] = c->L[r];
    return RE_OK;
}

int re_query_attempt_count(re_ctx* c, int64_t* n)
{
    if (!c || !n) return fail(c, RE_EINVAL, "NULL argument");
    *n = c->next_attempt;
    return RE_OK;
}

int re_query_exchange_log(re_ctx* c, re_xlog_rec* buf, int64_t cap, int64_t* n_out, int64_t* n_total)
{
    if (!c || cap < 0 || (cap > 0 && !buf) || !n_out) return fail(c, RE_EINVAL, "bad arguments");
    static_assert(sizeof(re_xlog_rec) == sizeof(XRec), "record layout");
    int64_t total = 0;
    int rc = d2h(c, &total, c->d.log_count, 1);
    if (rc) return rc;
    const int64_t avail = std::min(total, c->cfg.log_cap);
    const int64_t n = std::min(avail, cap);
    const int64_t first = total - n;  // oldest record copied
    for (int64_t k = 0; k < n;) {
        const int64_t pos = (first + k) % c->cfg.log_cap;
        const int64_t run = std::min(n - k, c->cfg.log_cap - pos);
        if ((rc = d2h(c, (XRec*)buf + k, c->d.log + pos, (size_t)run))) return rc;
        k += run;
    }
    *n_out = n;
    if (n_total) *n_total = total;
    return RE_OK;
}

int re_get_state(re_ctx* c, int r, double* x, double* v)
{
    if (!c || r < 0 || r >= c->R) return fail(c, RE_EINVAL, "bad replica index");
    const RepDev& rd = c->rep[r];
    const int N = rd.N;
    int rc;
    // velocities at the boundary include a factor still pending for the next
    // step (exchange rescale, thermostat rescale)
    double fac = 1.0;
    {
        int32_t ap = 0;
        if (c->ps.apend && (rc = d2h(c, &ap, c->ps.apend + r, 1))) return rc;
        if (c->pending_alpha || ap) {
            if ((rc = d2h(c, &fac, c->d.alpha + r, 1))) return rc;
        }
    }
    if (c->prec == RE_MIXED) {
        std::vector<int4> p(N);
        std::vector<float4> w(N);
        if ((rc = d2h(c, p.data(), c->d.posi[c->cur] + rd.base, N))) return rc;
        if ((rc = d2h(c, w.data(), c->d.velf + rd.base, N))) return rc;
        for (int k = 0; k < N; ++k) {
            const int i = p[k].w;
            if (i < 0 || i >= N) return fail(c, RE_EDEVICE, "corrupt atom id %d", i);
            if (x) {
                x[3 * i] = (double)p[k].x * rd.s;
                x[3 * i + 1] = (double)p[k].y * rd.s;
                x[3 * i + 2] = (double)p[k].z * rd.s;
            }
            if (v) {
                v[3 * i] = fac * w[k].x;
                v[3 * i + 1] = fac * w[k].y;
                v[3 * i + 2] = fac * w[k].z;
            }
        }
    } else {
        std::vector<double4> p(N), w(N);
        if ((rc = d2h(c, p.data(), c->d.posd[c->cur] + rd.base, N))) return rc;
        if ((rc = d2h(c, w.data(), c->d.veld + rd.base, N))) return rc;
        for (int k = 0; k < N; ++k) {
            const int i = (int)p[k].w;
            if (i < 0 || i >= N) return fail(c, RE_EDEVICE, "corrupt atom id %d", i);
            if (x) {
                x[3 * i] = p[k].x;
                x[3 * i + 1] = p[k].y;
                x[3 * i + 2] = p[k].z;
            }
            if (v) {
                v[3 * i] = fac * w[k].x;
                v[3 * i + 1] = fac * w[k].y;
                v[3 * i + 2] = fac * w[k].z;
            }
        }
    }
    return RE_OK;
}

int re_set_state(re_ctx* c, int r, const double* x, const double* v)
{
    if (!c || r < 0 || r >= c->R || !x || !v) return fail(c, RE_EINVAL, "bad arguments");
    int rc;
    if ((rc = upload_replica(c, r, x, v))) return rc;
    if ((rc = refresh_replicas(c, r, 1))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_overflow(c);
}

int re_compute_forces(re_ctx* c, int r, double* F, double* U)
{
    if (!c || r < 0 || r >= c->R) return fail(c, RE_EINVAL, "bad replica index");
    const bool f64 = c->prec == RE_FP64;
    StepArgs a = base_args(c);
    a.tab = c->ctF;
    a.blk_off = c->cF_start[r];
    HIPCHK(c, launch_force(f64, kQuery, c->d, a, c->cF_count[r], c->stream));
    const RepDev& rd = c->rep[r];
    std::vector<double> q(4 * (size_t)rd.N);
    int rc = d2h(c, q.data(), c->d.fq + 4 * (size_t)rd.base, q.size());
    if (rc) return rc;
    double u = 0;
    for (int i = 0; i < rd.N; ++i) {
        if (F) {
            F[3 * i] = q[4 * i];
            F[3 * i + 1] = q[4 * i + 1];
            F[3 * i + 2] = q[4 * i + 2];
        }
        u += q[4 * i + 3];
    }
    if (U) *U = 0.5 * u;
    return RE_OK;
}

int re_query_forces(re_ctx* c, int r, double* F)
{
    if (!c || r < 0 || r >= c->R || !F) return fail(c, RE_EINVAL, "bad arguments");
    const RepDev& rd = c->rep[r];
    const int N = rd.N;
    int rc;
    if (c->prec == RE_MIXED) {
        std::vector<int4> p(N);
        std::vector<float4> f(N);
        if ((rc = d2h(c, p.data(), c->d.posi[c->cur] + rd.base, N))) return rc;
        if ((rc = d2h(c, f.data(), c->d.frcf + rd.base, N))) return rc;
        for (int k = 0; k < N; ++k) {
            const int i = p[k].w;
            if (i < 0 || i >= N) return fail(c, RE_EDEVICE, "corrupt atom id %d", i);
            F[3 * i] = f[k].x;
            F[3 * i + 1] = f[k].y;
            F[3 * i + 2] = f[k].z;
        }
    } else {
        std::vector<double4> p(N), f(N);
        if ((rc = d2h(c, p.data(), c->d.posd[c->cur] + rd.base, N))) return rc;
        if ((rc = d2h(c, f.data(), c->d.frcd + rd.base, N))) return rc;
        for (int k = 0; k < N; ++k) {
            const int i = (int)p[k].w;
            if (i < 0 || i >= N) return fail(c, RE_EDEVICE, "corrupt atom id %d", i);
            F[3 * i] = f[k].x;
            F[3 * i + 1] = f[k].y;
            F[3 * i + 2] = f[k].z;
        }
    }
    return RE_OK;
}

int re_query_config(re_ctx* c, int* engine, int* threads_per_atom, int* team_size)
{
    if (!c) return fail(nullptr, RE_EINVAL, "ctx is NULL");
    const bool pers = c->form == RE_BATCHED && (c->engine == RE_PERSISTENT || c->xmode == RE_ASYNC);
    if (engine) *engine = pers ? RE_PERSISTENT : RE_LOCKSTEP;
    if (threads_per_atom) *threads_per_atom = c->cfg.tpa;
    if (team_size) *team_size = c->pers_ok && !c->team_of.empty() ? c->team_of[0] : 0;
    return RE_OK;
}

#ifdef RE_PHASE_TIMERS
// (instrumented build) the replica served by each workgroup of the launch
extern "C" int re_debug_team_rep(re_ctx* c, int32_t* out, int nmax)
{
    if (!c || !out || nmax < c->pnblk) return -1;
    return hipMemcpy(out, c->t_rep, (size_t)c->pnblk * 4, hipMemcpyDeviceToHost) == hipSuccess ? c->pnblk : -3;
}
#endif

int re_query_teams(re_ctx* c, int32_t* team)
{
    if (!c || !team) return fail(c, RE_EINVAL, "NULL argument");
    for (int r = 0; r < c->R; ++r) team[r] = c->pers_ok && (int)c->team_of.size() == c->R ? c->team_of[r] : 0;
    return RE_OK;
}

int re_query_lanes(re_ctx* c, int32_t* tpa)
{
    if (!c || !tpa) return fail(c, RE_EINVAL, "NULL argument");
    for (int r = 0; r < c->R; ++r) tpa[r] = c->tpa_r[r];
    return RE_OK;
}

int re_set_schedule(re_ctx* c, const int64_t* join, int64_t A)
{
    if (!c) return fail(nullptr, RE_EINVAL, "ctx is NULL");
    if (c->xmode != RE_ASYNC) return fail(c, RE_ESTATE, "schedules apply to asynchronous mode only");
    if (A < 0 || (A > 0 && !join)) return fail(c, RE_EINVAL, "bad schedule");
    const int R = c->R;
    std::vector<int64_t> steps(R);
    int rc = d2h(c, steps.data(), c->d.steps, R);
    if (rc) return rc;
    // each replica's join steps must increase strictly (a replica checks for
    // attempts after each of its steps)
    for (int64_t a = 0; a < A; ++a)
        for (int r = 0; r < R; ++r) {
            const int64_t prev = a ? join[(a - 1) * R + r] : steps[r];
            if (join[a * R + r] <= prev)
                return fail(c, RE_EINVAL, "join step of replica %d in attempt %lld must exceed %lld", r, (long long)a,
                            (long long)prev);
        }
    c->sched.assign(join, join + A * R);
    c->sched_A = A;
    return RE_OK;
}

int re_test_exchange(const double* U, const double* T, const int32_t* slot, int R, uint64_t seed, int64_t attempt,
                     int max_distance, uint8_t* decisions)
{
    if (!U || !T || !slot || !decisions || R < 1 || R > 4096 || max_distance < 1)
        return fail(nullptr, RE_EINVAL, "bad arguments");
    std::vector<int> seen(R, 0);
    for (int r = 0; r < R; ++r) {
        if (slot[r] < 0 || slot[r] >= R || seen[slot[r]]++) return fail(nullptr, RE_EINVAL, "slot is not a permutation");
    }
    double *dU = nullptr, *dT = nullptr;
    int32_t* ds = nullptr;
    uint8_t* dd = nullptr;
    hipError_t e = hipMalloc(&dU, R * 8);
    if (e == hipSuccess) e = hipMalloc(&dT, R * 8);
    if (e == hipSuccess) e = hipMalloc(&ds, R * 4);
    if (e == hipSuccess) e = hipMalloc(&dd, R);
    if (e == hipSuccess) e = hipMemcpy(dU, U, R * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dT, T, R * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ds, slot, R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_test_exchange(dU, dT, ds, R, seed, attempt, max_distance, dd, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess && R > 1) e = hipMemcpy(decisions, dd, R - 1, hipMemcpyDeviceToHost);
    (void)hipFree(dU);
    (void)hipFree(dT);
    (void)hipFree(ds);
    (void)hipFree(dd);
    if (e != hipSuccess) return fail(nullptr, RE_EDEVICE, "re_test_exchange: %s", hipGetErrorString(e));
    return RE_OK;
}

// Test hooks for the device random numbers: n Philox blocks of the given
// counters (4 words each) under key (key0, key1); and n normal triples
// (FP32 or FP64 Box-Muller) of the given counters under `seed`.
int re_test_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, int n, uint32_t* out)
{
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(nullptr, RE_EINVAL, "bad arguments");
    if (n == 0) return RE_OK;
    uint32_t *dc = nullptr, *dout = nullptr;
    hipError_t e = hipMalloc(&dc, 16 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&dout, 16 * (size_t)n);
    if (e == hipSuccess) e = hipMemcpy(dc, ctr, 16 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_test_philox(dc, key0, key1, n, dout, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, dout, 16 * (size_t)n, hipMemcpyDeviceToHost);
    (void)hipFree(dc);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(nullptr, RE_EDEVICE, "re_test_philox: %s", hipGetErrorString(e));
    return RE_OK;
}

int re_test_normals(int fp64, uint64_t seed, const uint32_t* ctr, int n, double* out)
{
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(nullptr, RE_EINVAL, "bad arguments");
    if (n == 0) return RE_OK;
    uint32_t* dc = nullptr;
    double* dout = nullptr;
    hipError_t e = hipMalloc(&dc, 16 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&dout, 24 * (size_t)n);
    if (e == hipSuccess) e = hipMemcpy(dc, ctr, 16 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_test_normals(fp64, seed, dc, n, dout, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, dout, 24 * (size_t)n, hipMemcpyDeviceToHost);
    (void)hipFree(dc);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(nullptr, RE_EDEVICE, "re_test_normals: %s", hipGetErrorString(e));
    return RE_OK;
}

// Timing of the dominant kernel (the fused force + integrate launch) with
// HIP events on the context's stream.  enable = 1 starts a window (up to
// 4096 launches are timed), 0 ends it; re_query_kernel_time reports the
// launches timed in the last window and their mean duration.
int re_profile(re_ctx* c, int enable)
{
    if (!c) return fail(nullptr, RE_EINVAL, "ctx is NULL");
    if (enable) {
        if (c->ev.empty()) {
            c->ev.resize(2 * 4096);
            for (auto& e : c->ev) HIPCHK(c, hipEventCreate(&e));
        }
        c->ev_used = 0;
        c->prof = true;
        return RE_OK;
    }
    c->prof = false;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0;
    for (int i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        tot += ms;
    }
    c->prof_ms = tot;
    c->prof_n = c->ev_used / 2;
    c->ev_used = 0;
    return RE_OK;
}

int re_query_kernel_time(re_ctx* c, double* mean_ms, int64_t* n)
{
    if (!c || !mean_ms || !n) return fail(c, RE_EINVAL, "NULL argument");
    *n = c->prof_n;
    *mean_ms = c->prof_n ? c->prof_ms / (double)c->prof_n : 0.0;
    return RE_OK;
}

void re_destroy(re_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (void* p : c->allocs) (void)hipFree(p);
    for (void* p : c->pinned) (void)hipHostFree(p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* re_last_error(const re_ctx* c)
{
    return c ? c->err.c_str() : g_noctx_error.c_str();
}

}  // extern "C"
