// C ABI of libsht (declared in include/sht.h): argument checks, the plan
// cache and the launch sequences of the inverse and forward transforms.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

#include "sht_internal.h"

using namespace sht;

namespace {

thread_local char g_last_hip_error[256] = "";

int hip_fail(hipError_t e, const char *where) {
    std::snprintf(g_last_hip_error, sizeof(g_last_hip_error), "%s: %s", where, hipGetErrorString(e));
    return SHT_ERR_HIP;
}

#define SHT_HIP(call, where)                          \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

struct DeviceState {
    EdgeTable E;
};

std::mutex g_mu;
std::map<int, DeviceState> g_devices;
std::map<std::tuple<int, int>, Plan *> g_plans;              // (device, L)
std::map<std::tuple<int, int, int>, SpinPlan *> g_spin;      // (device, L, spin)

// Plans are built one at a time (g_build_mu), on a stream of the library's
// own per device, with g_mu held only to look them up and to publish them: a
// first-use build waits for its own kernels, not for the caller's queued
// work, and transforms whose plans exist do not wait for it.  Lock order:
// g_build_mu before g_mu.
std::mutex g_build_mu;
std::map<int, hipStream_t> g_build_streams;

// ---- captured transforms ----
}  // namespace
struct sht_graph_s {
    int device;
    hipGraphExec_t exec;
    // the cached contraction table the captured kernels read (or none): its
    // use count in tab_sp->mtab_users[tab_cls] keeps it alive
    sht::SpinPlan *tab_sp;
    int tab_cls;
};
namespace {
std::mutex g_graph_mu;
std::set<sht_graph_s *> g_graphs;

// ---- stage tracing ----
struct TraceRec {
    int stage;
    hipEvent_t a, b;
};
bool g_trace_on = false;
thread_local bool t_capturing = false;  // inside sht_graph_create's capture
thread_local bool t_noalloc = false;    // inside sht_inverse_noalloc (no trace events)
std::mutex g_trace_mu;
std::vector<TraceRec> g_trace_pending;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pool_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs `launch` (returns hipError_t), bracketed by events when tracing is on.
template <typename F> hipError_t traced(int stage, hipStream_t st, F launch) {
    if (!g_trace_on || t_capturing || t_noalloc) return launch();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_trace_mu);
        a = pool_event();
        b = pool_event();
    }
    if (!a || !b) return launch();
    hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace_pending.push_back(TraceRec{stage, a, b});
    return hipSuccess;
}

int fft_size(int L) {
    int need = 4 * L - 3;
    if (need < 8) need = 8;
    return next_pow2(need);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t elem_bytes(int precision) { return precision == SHT_FP64 ? 8 : 4; }

// Workspace: two regions, each large enough for a set of order-major panels
// [L][4B][L] and for a B x L x N complex grid; the launch sequences below
// alternate between them.  Rows whose FFT buffer does not fit in LDS (FP64,
// L > 2048) add a third region: the split rows' scratch slots.
void regions(int L, int batch, int precision, size_t &ra, size_t &rb) {
    const size_t T = elem_bytes(precision);
    const size_t C = 4 * (size_t)batch, N = 2 * (size_t)L - 1;
    const size_t panel = (size_t)L * C * L * T;
    const size_t grid = (size_t)batch * L * 2 * (size_t)L * 2 * T;  // rings of ring_len = 2L (>= N)
    ra = align256(panel > grid ? panel : grid);
    rb = ra;
}
size_t split_region(int L, int precision) {
    const int M = fft_size(L), cb = 2 * (int)elem_bytes(precision);
    return rows_split(M, cb) ? align256((size_t)kSplitSlots * M * cb) : 0;
}
size_t workspace_total(int L, int batch, int precision) {
    size_t ra, rb;
    regions(L, batch, precision, ra, rb);
    return ra + rb + split_region(L, precision);
}

int check_args(int L, int spin, int batch, int sampling, int precision) {
    if (sampling != SHT_SAMPLING_MW) return SHT_ERR_UNSUPPORTED;
    if (precision != SHT_FP64 && precision != SHT_FP32 && precision != SHT_BF16X3) return SHT_ERR_UNSUPPORTED;
    if (L < 1 || L > SHT_L_MAX) return SHT_ERR_INVALID_ARG;
    if (spin <= -L || spin >= L) return SHT_ERR_INVALID_ARG;
    if (batch < 1 || batch > SHT_BATCH_MAX) return SHT_ERR_INVALID_ARG;
    return SHT_OK;
}

int get_device_state(int dev, hipStream_t st, DeviceState **out) {
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_devices.find(dev);
        if (it != g_devices.end()) { *out = &it->second; return SHT_OK; }
    }
    DeviceState ds;
    ds.E.lmax = SHT_L_MAX;
    const size_t n = (size_t)SHT_L_MAX * (SHT_L_MAX + 1) / 2;
    if (hipMalloc(&ds.E.mant, n * sizeof(double)) != hipSuccess) return SHT_ERR_OOM;
    if (hipMalloc(&ds.E.expo, n * sizeof(int)) != hipSuccess) { (void)hipFree(ds.E.mant); return SHT_ERR_OOM; }
    SHT_HIP(launch_edge_table(ds.E, st), "edge table");
    SHT_HIP(hipStreamSynchronize(st), "edge table sync");
    std::lock_guard<std::mutex> lock(g_mu);
    auto res = g_devices.emplace(dev, ds);
    *out = &res.first->second;
    return SHT_OK;
}

template <typename T> int alloc_fft(FftTables<T> &ft, int L) {
    using C = typename CT<T>::type;
    ft.L = L;
    ft.N = 2 * L - 1;
    ft.M = fft_size(L);
    ft.logM = ilog2(ft.M);
    const size_t nptw = (size_t)fft_pass_offset(ft.logM, fft_npass(ft.logM));
    // split rows (two M/2-point halves) also need the M/2-point pass twiddles
    const bool split = rows_split(ft.M, 2 * (int)sizeof(T));
    const size_t nptwh = split ? (size_t)fft_pass_offset(ft.logM - 1, fft_npass(ft.logM - 1)) : 0;
    const size_t n = (size_t)ft.M + 2 * (size_t)ft.N + 2 * (size_t)ft.N + nptw + 3 * (size_t)ft.M + nptwh;
    C *base = nullptr;
    if (hipMalloc(&base, n * sizeof(C)) != hipSuccess) return SHT_ERR_OOM;
    ft.tw = base;
    ft.e2n = ft.tw + ft.M;
    ft.cha = ft.e2n + 2 * ft.N;
    ft.chb = ft.cha + ft.N;
    ft.ptw = ft.chb + ft.N;
    ft.h_ip = ft.ptw + nptw;
    ft.h_fd = ft.h_ip + ft.M;
    ft.h_fk = ft.h_fd + ft.M;
    ft.ptwh = split ? ft.h_fk + ft.M : nullptr;
    return SHT_OK;
}

int get_plan(int dev, int L, hipStream_t st, Plan **out) {
    auto key = std::make_tuple(dev, L);
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) { *out = it->second; return SHT_OK; }
    }
    Plan *p = new Plan();
    p->device = dev;
    p->L = L;
    int rc = alloc_fft(p->f64, L);
    if (rc == SHT_OK) rc = alloc_fft(p->f32, L);
    if (rc != SHT_OK) { delete p; return rc; }
    if (hipMalloc(&p->rec.ri, (size_t)L * L * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->rec.rf, (size_t)L * L * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->rec.fab, (size_t)L * L * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->rec.jti, (size_t)(L + 2 * kTabPad) * L * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->rec.jtf, (size_t)(L + 2 * kTabPad) * L * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->rec.cl, (size_t)L * sizeof(double)) != hipSuccess) {
        delete p;
        return SHT_ERR_OOM;
    }
    SHT_HIP(hipMemsetAsync(p->rec.jti, 0, (size_t)(L + 2 * kTabPad) * L * sizeof(double2), st), "table padding");
    SHT_HIP(hipMemsetAsync(p->rec.jtf, 0, (size_t)(L + 2 * kTabPad) * L * sizeof(double2), st), "table padding");
    p->rec.jti += (size_t)kTabPad * L;
    p->rec.jtf += (size_t)kTabPad * L;
    SHT_HIP(launch_rec_tables(L, p->rec, st), "recursion tables");
    if (build_contract_schedules(L, p->rec) != 0) {
        delete p;
        return SHT_ERR_OOM;
    }
    SHT_HIP(launch_fft_tables<double>(p->f64, nullptr, st), "fft tables f64");
    SHT_HIP(launch_fft_tables<float>(p->f32, &p->f64, st), "fft tables f32");
    SHT_HIP(prepare_row_kernels<double>(p->f64), "row kernel attributes f64");
    SHT_HIP(prepare_row_kernels<float>(p->f32), "row kernel attributes f32");
    SHT_HIP(hipStreamSynchronize(st), "plan sync");
    std::lock_guard<std::mutex> lock(g_mu);
    g_plans[key] = p;
    *out = p;
    return SHT_OK;
}

int get_spin_plan(int dev, int L, int spin, const DeviceState *ds, const Plan *plan, hipStream_t st,
                  SpinPlan **out) {
    auto key = std::make_tuple(dev, L, spin);
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_spin.find(key);
        if (it != g_spin.end()) { *out = it->second; return SHT_OK; }
    }
    SpinPlan *sp = new SpinPlan();
    sp->device = dev;
    sp->L = L;
    sp->spin = spin;
    // one block: wi, wf (FP64) then wi32, wf32 (FP32), each L rows of L
    // between kTabPad zero rows
    const size_t n = (size_t)(L + 2 * kTabPad) * L, pad = (size_t)kTabPad * L;
    const size_t bytes = n * (2 * sizeof(double) + 2 * sizeof(float));
    char *blk = nullptr;
    if (hipMalloc(&blk, bytes) != hipSuccess) { delete sp; return SHT_ERR_OOM; }
    SHT_HIP(hipMemsetAsync(blk, 0, bytes, st), "table padding");
    sp->wi = (double *)blk + pad;
    sp->wf = (double *)blk + n + pad;
    sp->wi32 = (float *)((double *)blk + 2 * n) + pad;
    sp->wf32 = (float *)((double *)blk + 2 * n) + n + pad;
    SHT_HIP(launch_spin_tables(ds->E, plan->rec, *sp, st), "spin tables");
    SHT_HIP(hipStreamSynchronize(st), "spin plan sync");
    std::lock_guard<std::mutex> lock(g_mu);
    g_spin[key] = sp;
    *out = sp;
    return SHT_OK;
}

// the resident plans of (dev, L, spin), if all exist (g_mu held)
bool find_ready(int dev, int L, int spin, DeviceState **ds, Plan **plan, SpinPlan **sp) {
    auto d = g_devices.find(dev);
    auto p = g_plans.find(std::make_tuple(dev, L));
    auto q = g_spin.find(std::make_tuple(dev, L, spin));
    if (d == g_devices.end() || p == g_plans.end() || q == g_spin.end()) return false;
    *ds = &d->second;
    *plan = p->second;
    *sp = q->second;
    return true;
}

// the library's build stream of the device (g_build_mu held)
int build_stream(int dev, hipStream_t *out) {
    auto it = g_build_streams.find(dev);
    if (it == g_build_streams.end()) {
        hipStream_t s = nullptr;
        SHT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "plan build stream");
        it = g_build_streams.emplace(dev, s).first;
    }
    *out = it->second;
    return SHT_OK;
}

int prepare(int L, int spin, DeviceState **ds, Plan **plan, SpinPlan **sp) {
    int dev = 0;
    SHT_HIP(hipGetDevice(&dev), "hipGetDevice");
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (find_ready(dev, L, spin, ds, plan, sp)) return SHT_OK;
    }
    std::lock_guard<std::mutex> build(g_build_mu);
    hipStream_t bs = nullptr;
    int rc = build_stream(dev, &bs);
    if (rc != SHT_OK) return rc;
    rc = get_device_state(dev, bs, ds);
    if (rc != SHT_OK) return rc;
    rc = get_plan(dev, L, bs, plan);
    if (rc != SHT_OK) return rc;
    return get_spin_plan(dev, L, spin, *ds, *plan, bs, sp);
}

bool misaligned(const void *p, size_t a) { return ((uintptr_t)p) % a != 0; }

int check_buffers(int L, int batch, int precision, const void *in, const void *out, const void *ws,
                  size_t ws_bytes) {
    if (!in || !out || !ws) return SHT_ERR_INVALID_ARG;
    const size_t ca = 2 * elem_bytes(precision);
    if (misaligned(in, ca) || misaligned(out, ca) || misaligned(ws, 256)) return SHT_ERR_ALIGNMENT;
    if (ws_bytes < workspace_total(L, batch, precision)) return SHT_ERR_WORKSPACE;
    return SHT_OK;
}

// Real maps: the map is real (element-aligned), the coefficients complex.
int check_buffers_real(bool inverse, int L, int batch, int precision, const void *in, const void *out,
                       const void *ws, size_t ws_bytes) {
    if (!in || !out || !ws) return SHT_ERR_INVALID_ARG;
    const size_t e = elem_bytes(precision);
    const void *flm = inverse ? in : out, *map = inverse ? out : in;
    if (misaligned(flm, 2 * e) || misaligned(map, e) || misaligned(ws, 256)) return SHT_ERR_ALIGNMENT;
    if (ws_bytes < workspace_total(L, batch, precision)) return SHT_ERR_WORKSPACE;
    return SHT_OK;
}

// One spin's maps within a call: `B` maps, stored after the maps of the
// earlier segments; their contraction columns follow those segments' too.
// flip: the segment follows one of the opposite spin and shares its
// contraction factors, d^l_{m',s}(pi/2) = (-1)^{l+m'} d^l_{m',-s}(pi/2)
// (Eq. (wignerd_sym6)); the layout and theta stages apply the signs.
struct Seg {
    int spin, B;
    const SpinPlan *sp;
    int flip;
};
constexpr int kMaxSegs = SHT_MULTI_SEG_MAX;

// Marks each segment of spin -s that directly follows one of spin s != 0 to
// share that segment's contraction (one column range, one Wigner
// generation per column block for both).
void pair_segments(int nseg, Seg *seg) {
    for (int k = 0; k < nseg; ++k) seg[k].flip = 0;
    for (int k = 0; k + 1 < nseg; ++k) {
        if (seg[k].spin != 0 && !seg[k].flip && seg[k + 1].spin == -seg[k].spin) {
            seg[k + 1].flip = 1;
            ++k;
        }
    }
}

// The contraction in the path's own precision, or as BF16x3 on FP32 data,
// over every segment's columns in one launch (a flipped segment joins the
// column range of the segment before it).
template <typename T>
hipError_t contract(int mode, bool bf16x3, int L, int nq, int nseg, const Seg *seg, const T *X, T *Y,
                    const DeviceState *ds, const RecTables &rec, hipStream_t st) {
    ContractSeg cs[kMaxSegs];
    int n = 0;
    for (int k = 0; k < nseg; ++k) {
        if (seg[k].flip && n > 0) cs[n - 1].ncol += nq * seg[k].B;
        else cs[n++] = ContractSeg{nq * seg[k].B, seg[k].sp};
    }
    nseg = n;
    if constexpr (sizeof(T) == 4) {
        if (bf16x3) return launch_contract_bf16x3(mode, L, nseg, cs, X, Y, ds->E, rec, st);
    }
    return launch_contract<T>(mode, L, nseg, cs, X, Y, ds->E, rec, st);
}

// The segment table of the layout and theta kernels: the maps of segment k
// follow those of the segments before it, in the caller's buffers, the rings
// and the panel columns.
SpinSegs spin_segs(int nq, int nseg, const Seg *seg) {
    SpinSegs sg{};
    sg.n = nseg;
    for (int k = 0; k < nseg; ++k) {
        sg.seg[k] = SpinSeg{seg[k].spin, seg[k].B, sg.batch, nq * sg.batch, seg[k].flip};
        sg.batch += seg[k].B;
    }
    return sg;
}

// real: spin-0 real maps; only the orders m >= 0 are carried (2 columns per
// map, L theta rows), and the phi stages read / write real rings.
// Every stage runs once over all maps: the layout and theta kernels look up
// each map's segment (its spin enters the phases and the parity extension),
// the contraction takes one column range per segment or spin pair.
template <typename T>
int run_inverse(int L, int nseg, const Seg *seg, bool bf16x3, bool real, const FftTables<T> &ft,
                const RecTables &rec, const DeviceState *ds, const void *flm, void *map, void *ws, hipStream_t st) {
    int batch = 0;
    for (int k = 0; k < nseg; ++k) batch += seg[k].B;
    size_t ra, rb;
    regions(L, batch, sizeof(T) == 8 ? SHT_FP64 : SHT_FP32, ra, rb);
    unsigned char *w = (unsigned char *)ws;
    T *P = (T *)w;            // region A: layout panels, later the theta-stage output
    T *R = (T *)(w + ra);     // region B: contraction output
    void *scr = w + ra + rb;  // split-row scratch (L > 2048, FP64)
    const int nq = real ? 2 : 4, Cn = nq * batch;
    const SpinSegs lsg = spin_segs(nq, nseg, seg);
    SHT_HIP(traced(SHT_STAGE_LAYOUT_IN, st, [&] { return launch_layout_in<T>(L, lsg, Cn, real, flm, P, st); }),
            "layout_in");
    SHT_HIP(traced(SHT_STAGE_CONTRACT_INV, st,
                   [&] { return contract<T>(kInverse, bf16x3, L, nq, nseg, seg, P, R, ds, rec, st); }),
            "contract inverse");
    // theta stage writes g_mu(theta_t) straight into the rings over mu that
    // the phi stage reads (region A; the panels are no longer needed)
    SHT_HIP(traced(SHT_STAGE_THETA_INV, st,
                   [&] { return launch_theta_inv<T>(ft, lsg, Cn, real, R, P, scr, st); }),
            "theta inverse");
    SHT_HIP(traced(SHT_STAGE_PHI_INV, st,
                   [&] {
                       return real ? launch_phi_inv_real<T>(ft, batch, (const void *)P, (T *)map, scr, st)
                                   : launch_phi_inv<T>(ft, batch, ring_len(L, false), (const void *)P, map, scr, st);
                   }),
            "phi inverse");
    return SHT_OK;
}

template <typename T>
int run_forward(int L, int nseg, const Seg *seg, bool bf16x3, bool real, const FftTables<T> &ft,
                const RecTables &rec, const DeviceState *ds, const void *map, void *flm, void *ws, hipStream_t st) {
    int batch = 0;
    for (int k = 0; k < nseg; ++k) batch += seg[k].B;
    size_t ra, rb;
    regions(L, batch, sizeof(T) == 8 ? SHT_FP64 : SHT_FP32, ra, rb);
    unsigned char *w = (unsigned char *)ws;
    void *Q = (void *)(w + ra);   // region B: phi-stage output (rings over mu)
    T *X = (T *)w;                // region A: weighted theta coefficients
    void *scr = w + ra + rb;      // split-row scratch (L > 2048, FP64)
    const int nq = real ? 2 : 4, Cn = nq * batch;
    SHT_HIP(traced(SHT_STAGE_PHI_FWD, st,
                   [&] {
                       return real ? launch_phi_fwd_real<T>(ft, batch, (const T *)map, Q, scr, st)
                                   : launch_phi_fwd<T>(ft, batch, ring_len(L, false), map, Q, scr, st);
                   }),
            "phi forward");
    // the theta stage reads its two orders as columns of the rings in place
    const SpinSegs lsg = spin_segs(nq, nseg, seg);
    SHT_HIP(traced(SHT_STAGE_THETA_FWD, st,
                   [&] { return launch_theta_fwd<T>(ft, lsg, Cn, real, Q, X, scr, st); }),
            "theta forward");
    T *R = (T *)(w + ra);
    SHT_HIP(traced(SHT_STAGE_CONTRACT_FWD, st,
                   [&] { return contract<T>(kForward, bf16x3, L, nq, nseg, seg, X, R, ds, rec, st); }),
            "contract forward");
    SHT_HIP(traced(SHT_STAGE_LAYOUT_OUT, st, [&] { return launch_layout_out<T>(L, lsg, Cn, real, R, flm, st); }),
            "layout_out");
    return SHT_OK;
}

// The transform of nseg spin segments (spins[k], batches[k] maps each, in
// that order in the caller's buffers).
int transform_segs(bool inverse, bool real, int L, int nseg, const int *spins, const int *batches, int sampling,
                   int precision, const void *in, void *out, void *workspace, size_t ws_bytes, void *stream) {
    if (nseg < 1 || nseg > kMaxSegs || !spins || !batches) return SHT_ERR_INVALID_ARG;
    int batch = 0;
    for (int k = 0; k < nseg; ++k) {
        if (batches[k] < 1) return SHT_ERR_INVALID_ARG;
        batch += batches[k];
        if (batch > SHT_BATCH_MAX) return SHT_ERR_INVALID_ARG;
        const int rc = check_args(L, spins[k], batches[k], sampling, precision);
        if (rc != SHT_OK) return rc;
        if (real && spins[k] != 0) return SHT_ERR_INVALID_ARG;
    }
    int rc = real ? check_buffers_real(inverse, L, batch, precision, in, out, workspace, ws_bytes)
                  : check_buffers(L, batch, precision, in, out, workspace, ws_bytes);
    if (rc != SHT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    DeviceState *ds = nullptr;
    Plan *plan = nullptr;
    Seg seg[kMaxSegs];
    for (int k = 0; k < nseg; ++k) {
        SpinPlan *sp;
        rc = prepare(L, spins[k], &ds, &plan, &sp);
        if (rc != SHT_OK) return rc;
        seg[k] = Seg{spins[k], batches[k], sp, 0};
    }
    if (!real) pair_segments(nseg, seg);
    const bool bf = precision == SHT_BF16X3;
    if (precision == SHT_FP64) {
        return inverse ? run_inverse<double>(L, nseg, seg, false, real, plan->f64, plan->rec, ds, in, out,
                                             workspace, st)
                       : run_forward<double>(L, nseg, seg, false, real, plan->f64, plan->rec, ds, in, out,
                                             workspace, st);
    }
    return inverse ? run_inverse<float>(L, nseg, seg, bf, real, plan->f32, plan->rec, ds, in, out, workspace, st)
                   : run_forward<float>(L, nseg, seg, bf, real, plan->f32, plan->rec, ds, in, out, workspace, st);
}

int transform(bool inverse, bool real, int L, int spin, int batch, int sampling, int precision, const void *in,
              void *out, void *workspace, size_t ws_bytes, void *stream) {
    return transform_segs(inverse, real, L, 1, &spin, &batch, sampling, precision, in, out, workspace, ws_bytes,
                          stream);
}

// ---- the inverse that allocates nothing (sht_inverse_noalloc) ----
// Its workspace: one static array per device, held until the process ends.
// In host code `scratch` names a host-side stand-in; the device address of
// each device's copy comes from hipGetSymbolAddress (scratch_on) and only that
// address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SHT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up on the first
// call on that device (with it current) and kept.
int scratch_on(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return SHT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch address");
        if (!p) return hip_fail(hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SHT_OK;
}

// The resident plans of (current device, L, spin), or SHT_ERR_NOT_READY:
// nothing is built here.
int find_plans(int dev, int L, int spin, DeviceState **ds, Plan **plan, SpinPlan **sp) {
    std::lock_guard<std::mutex> lock(g_mu);
    return find_ready(dev, L, spin, ds, plan, sp) ? SHT_OK : SHT_ERR_NOT_READY;
}

}  // namespace

extern "C" {

int sht_inverse_noalloc(int L, int spin, int batch, int sampling, int precision, const void *flm, void *map,
                        void *stream) {
    int rc = check_args(L, spin, batch, sampling, precision);
    if (rc != SHT_OK) return rc;
    if (!flm || !map) return SHT_ERR_INVALID_ARG;
    const size_t ca = 2 * elem_bytes(precision);
    if (misaligned(flm, ca) || misaligned(map, ca)) return SHT_ERR_ALIGNMENT;
    if (workspace_total(L, batch, precision) > (size_t)SHT_NOALLOC_SCRATCH_BYTES) return SHT_ERR_WORKSPACE;
    int dev = 0;
    SHT_HIP(hipGetDevice(&dev), "hipGetDevice");
    void *ws = nullptr;
    rc = scratch_on(dev, &ws);
    if (rc != SHT_OK) return rc;
    DeviceState *ds;
    Plan *plan;
    SpinPlan *sp;
    rc = find_plans(dev, L, spin, &ds, &plan, &sp);
    if (rc != SHT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const Seg one{spin, batch, sp, 0};
    t_noalloc = true;
    rc = precision == SHT_FP64
             ? run_inverse<double>(L, 1, &one, false, false, plan->f64, plan->rec, ds, flm, map, ws, st)
             : run_inverse<float>(L, 1, &one, precision == SHT_BF16X3, false, plan->f32, plan->rec, ds, flm, map, ws,
                                  st);
    t_noalloc = false;
    return rc;
}

size_t sht_workspace_bytes(int L, int spin, int batch, int sampling, int precision) {
    if (check_args(L, spin, batch, sampling, precision) != SHT_OK) return 0;
    return workspace_total(L, batch, precision);
}

int sht_inverse(int L, int spin, int batch, int sampling, int precision, const void *flm, void *map,
                void *workspace, size_t ws_bytes, void *stream) {
    return transform(true, false, L, spin, batch, sampling, precision, flm, map, workspace, ws_bytes, stream);
}

int sht_forward(int L, int spin, int batch, int sampling, int precision, const void *map, void *flm,
                void *workspace, size_t ws_bytes, void *stream) {
    return transform(false, false, L, spin, batch, sampling, precision, map, flm, workspace, ws_bytes, stream);
}

int sht_inverse_multi(int L, int nseg, const int *spins, const int *batches, int sampling, int precision,
                      const void *flm, void *map, void *workspace, size_t ws_bytes, void *stream) {
    return transform_segs(true, false, L, nseg, spins, batches, sampling, precision, flm, map, workspace, ws_bytes,
                          stream);
}

int sht_forward_multi(int L, int nseg, const int *spins, const int *batches, int sampling, int precision,
                      const void *map, void *flm, void *workspace, size_t ws_bytes, void *stream) {
    return transform_segs(false, false, L, nseg, spins, batches, sampling, precision, map, flm, workspace, ws_bytes,
                          stream);
}

int sht_inverse_real(int L, int batch, int sampling, int precision, const void *flm, void *map, void *workspace,
                     size_t ws_bytes, void *stream) {
    return transform(true, true, L, 0, batch, sampling, precision, flm, map, workspace, ws_bytes, stream);
}

int sht_forward_real(int L, int batch, int sampling, int precision, const void *map, void *flm, void *workspace,
                     size_t ws_bytes, void *stream) {
    return transform(false, true, L, 0, batch, sampling, precision, map, flm, workspace, ws_bytes, stream);
}

int sht_forward_triangular(int L, int spin, int batch, int sampling, int precision, const void *map, void *flm,
                           void *workspace, size_t ws_bytes, void *stream) {
    int rc = check_args(L, spin, batch, sampling, precision);
    if (rc != SHT_OK) return rc;
    if (precision != SHT_FP64 || L > SHT_TRI_L_MAX) return SHT_ERR_UNSUPPORTED;
    rc = check_buffers(L, batch, precision, map, flm, workspace, ws_bytes);
    if (rc != SHT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    DeviceState *ds;
    Plan *plan;
    SpinPlan *sp;
    rc = prepare(L, spin, &ds, &plan, &sp);
    if (rc != SHT_OK) return rc;
    size_t ra, rb;
    regions(L, batch, precision, ra, rb);
    unsigned char *w = (unsigned char *)workspace;
    void *A = (void *)w;         // phi-stage output, later the torus coefficients
    void *Bq = (void *)(w + ra); // the same rows over t
    const FftTables<double> &ft = plan->f64;
    SHT_HIP(launch_phi_fwd<double>(ft, batch, ft.N, map, A, nullptr, st), "phi forward");
    SHT_HIP(launch_transpose<double>(batch, L, ft.N, A, Bq, st), "transpose");
    SHT_HIP(launch_theta_dft<double>(ft, spin, batch, Bq, A, st), "theta dft");
    SHT_HIP(launch_tri_solve(L, spin, batch, A, flm, ds->E, *sp, plan->rec, st), "triangular solve");
    return SHT_OK;
}

int sht_forward_lstsq(int L, int spin, int batch, int sampling, int precision, const void *map, void *flm,
                      void *workspace, size_t ws_bytes, void *stream) {
    int rc = check_args(L, spin, batch, sampling, precision);
    if (rc != SHT_OK) return rc;
    if (precision != SHT_FP64 || L > SHT_TRI_L_MAX) return SHT_ERR_UNSUPPORTED;
    rc = check_buffers(L, batch, precision, map, flm, workspace, ws_bytes);
    if (rc != SHT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    DeviceState *ds;
    Plan *plan;
    SpinPlan *sp;
    rc = prepare(L, spin, &ds, &plan, &sp);
    if (rc != SHT_OK) return rc;
    size_t ra, rb;
    regions(L, batch, precision, ra, rb);
    unsigned char *w = (unsigned char *)workspace;
    void *A = (void *)w;         // phi-stage output, later the torus coefficients
    void *Bq = (void *)(w + ra); // the same rows over t
    const FftTables<double> &ft = plan->f64;
    SHT_HIP(launch_phi_fwd<double>(ft, batch, ft.N, map, A, nullptr, st), "phi forward");
    SHT_HIP(launch_transpose<double>(batch, L, ft.N, A, Bq, st), "transpose");
    SHT_HIP(launch_theta_dft<double>(ft, spin, batch, Bq, A, st), "theta dft");
    SHT_HIP(launch_tri_lstsq(L, spin, batch, A, flm, ds->E, *sp, plan->rec, st), "least-squares solve");
    return SHT_OK;
}

int sht_spin_pair(int L, int spin, int batch, int precision, const void *flm_s, void *flm_ms, void *stream) {
    int rc = check_args(L, spin, batch, SHT_SAMPLING_MW, precision);
    if (rc != SHT_OK) return rc;
    if (!flm_s || !flm_ms) return SHT_ERR_INVALID_ARG;
    if (flm_s == flm_ms) return SHT_ERR_INVALID_ARG;
    const size_t ca = 2 * elem_bytes(precision);
    if (misaligned(flm_s, ca) || misaligned(flm_ms, ca)) return SHT_ERR_ALIGNMENT;
    hipStream_t st = (hipStream_t)stream;
    if (precision == SHT_FP64) SHT_HIP(launch_spin_pair<double>(L, spin, batch, flm_s, flm_ms, st), "spin pair");
    else SHT_HIP(launch_spin_pair<float>(L, spin, batch, flm_s, flm_ms, st), "spin pair");
    return SHT_OK;
}

int sht_plan_tables(int L, int spin, int precision, int enable, void *stream) {
    int rc = check_args(L, spin, 1, SHT_SAMPLING_MW, precision);
    if (rc != SHT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    DeviceState *ds;
    Plan *plan;
    SpinPlan *sp;
    rc = prepare(L, spin, &ds, &plan, &sp);
    if (rc != SHT_OK) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    const bool f64 = precision == SHT_FP64;
    void **slot = f64 ? (void **)&sp->mtab64 : (void **)&sp->mtab32;
    if (!enable) {
        if (sp->mtab_users[f64 ? 1 : 0] > 0) return SHT_ERR_BUSY;  // a captured graph streams it
        if (*slot) {
            SHT_HIP(hipStreamSynchronize(st), "table release sync");
            SHT_HIP(hipFree(*slot), "table free");
            *slot = nullptr;
        }
        return SHT_OK;
    }
    if (*slot) return SHT_OK;
    const size_t bytes = (size_t)L * L * L * (f64 ? sizeof(double) : sizeof(float));
    if (hipMalloc(slot, bytes) != hipSuccess) {
        *slot = nullptr;
        return SHT_ERR_OOM;
    }
    SHT_HIP(launch_mtable(L, f64 ? 1 : 0, ds->E, plan->rec, *sp, st), "contraction table");
    SHT_HIP(hipStreamSynchronize(st), "contraction table sync");
    return SHT_OK;
}

int sht_plan_warmup(int L, int spin, int sampling, int precision, void *stream) {
    int rc = check_args(L, spin, 1, sampling, precision);
    if (rc != SHT_OK) return rc;
    DeviceState *ds;
    Plan *plan;
    SpinPlan *sp;
    return prepare(L, spin, &ds, &plan, &sp);
}

size_t sht_error_workspace_bytes(void) { return error_workspace_bytes(); }

int sht_error_metrics(int precision, size_t n, const void *ref, const void *val, double *out, void *workspace,
                      size_t ws_bytes, void *stream) {
    if (precision != SHT_FP64 && precision != SHT_FP32 && precision != SHT_BF16X3) return SHT_ERR_UNSUPPORTED;
    if (!out || !workspace || (n > 0 && (!ref || !val))) return SHT_ERR_INVALID_ARG;
    const size_t esz = precision == SHT_FP64 ? 16 : 8;
    if (n > ((size_t)1 << 40) / esz) return SHT_ERR_INVALID_ARG;
    if (misaligned(workspace, 256) || misaligned(out, 8) || misaligned(ref, esz / 2) || misaligned(val, esz / 2))
        return SHT_ERR_ALIGNMENT;
    if (ws_bytes < error_workspace_bytes()) return SHT_ERR_WORKSPACE;
    SHT_HIP(launch_error_metrics(precision == SHT_FP64, ref, val, n, out, workspace, (hipStream_t)stream),
            "error metrics");
    return SHT_OK;
}

int sht_tile_set(int L, int columns, int precision, int tile) {
    if (L < 1 || L > SHT_L_MAX || columns < 1 || columns > 4 * SHT_BATCH_MAX) return SHT_ERR_INVALID_ARG;
    if (precision != SHT_FP64 && precision != SHT_FP32 && precision != SHT_BF16X3) return SHT_ERR_UNSUPPORTED;
    const bool wide = tile == 128 && precision == SHT_FP32;  // the 128-column tile is FP32 only
    if (tile != 0 && tile != 16 && tile != 32 && tile != 64 && !wide) return SHT_ERR_INVALID_ARG;
    set_contract_tile(L, columns, contract_precision_class(precision == SHT_FP64, precision == SHT_BF16X3), tile);
    return SHT_OK;
}

int sht_tune(int L, int spin, int batch, int precision, void *workspace, size_t ws_bytes, void *stream,
             int *tile_out) {
    int rc = check_args(L, spin, batch, SHT_SAMPLING_MW, precision);
    if (rc != SHT_OK) return rc;
    if (!workspace) return SHT_ERR_INVALID_ARG;
    if (misaligned(workspace, 256)) return SHT_ERR_ALIGNMENT;
    size_t ra, rb;
    regions(L, batch, precision, ra, rb);
    if (ws_bytes < workspace_total(L, batch, precision)) return SHT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    DeviceState *ds;
    Plan *plan;
    SpinPlan *sp;
    rc = prepare(L, spin, &ds, &plan, &sp);
    if (rc != SHT_OK) return rc;
    const int C = 4 * batch;
    const bool f64 = precision == SHT_FP64, bf = precision == SHT_BF16X3;
    const int pc = contract_precision_class(f64, bf);
    unsigned char *w = (unsigned char *)workspace;
    // region A as the contraction input (zeroed: the timing does not depend
    // on the values), region B as its output
    SHT_HIP(hipMemsetAsync(w, 0, ra, st), "tune clear");
    hipEvent_t e0, e1;
    SHT_HIP(hipEventCreate(&e0), "tune event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(hipErrorOutOfMemory, "tune event");
    }
    const int tiles[4] = {16, 32, 64, 128};
    const int ntiles = precision == SHT_FP32 ? 4 : 3;
    int best = 0;
    float best_ms = 0.0f;
    rc = SHT_OK;
    for (int i = 0; i < ntiles && rc == SHT_OK; ++i) {
        set_contract_tile(L, C, pc, tiles[i]);
        float ms = 0.0f;
        for (int rep = 0; rep < 3 && rc == SHT_OK; ++rep) {  // rep 0 warms up
            hipError_t e = hipEventRecord(e0, st);
            const Seg one{spin, batch, sp, 0};
            for (int mode = 0; mode < 2 && e == hipSuccess; ++mode) {
                if (f64)
                    e = contract<double>(mode, false, L, 4, 1, &one, (const double *)w, (double *)(w + ra), ds,
                                         plan->rec, st);
                else
                    e = contract<float>(mode, bf, L, 4, 1, &one, (const float *)w, (float *)(w + ra), ds, plan->rec,
                                        st);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) rc = hip_fail(e, "tune run");
            if (rep > 0) ms += t;
        }
        if (rc == SHT_OK && (best == 0 || ms < best_ms)) {
            best = tiles[i];
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_contract_tile(L, C, pc, rc == SHT_OK ? best : 0);
    if (rc == SHT_OK && tile_out) *tile_out = best;
    return rc;
}

int sht_graph_create(int L, int spin, int batch, int sampling, int precision, const void *flm_in, void *map,
                     void *flm_out, void *workspace, size_t ws_bytes, void *stream, sht_graph *out) {
    if (!out) return SHT_ERR_INVALID_ARG;
    *out = nullptr;
    int rc = check_args(L, spin, batch, sampling, precision);
    if (rc != SHT_OK) return rc;
    rc = check_buffers(L, batch, precision, flm_in, map, workspace, ws_bytes);
    if (rc == SHT_OK) rc = check_buffers(L, batch, precision, map, flm_out, workspace, ws_bytes);
    if (rc != SHT_OK) return rc;
    // the plan is built (and synchronised) before the capture starts, so the
    // captured sequence is kernel launches only
    rc = sht_plan_warmup(L, spin, sampling, precision, stream);
    if (rc != SHT_OK) return rc;
    int dev = 0;
    SHT_HIP(hipGetDevice(&dev), "graph device");
    // a cached table that the captured contraction will read stays alive
    // until the graph is destroyed (sht_plan_tables refuses to free it)
    SpinPlan *tab_sp = nullptr;
    const int tab_cls = precision == SHT_FP64 ? 1 : 0;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_spin.find(std::make_tuple(dev, L, spin));
        if (it != g_spin.end() && (tab_cls ? (void *)it->second->mtab64 : (void *)it->second->mtab32)) {
            tab_sp = it->second;
            ++tab_sp->mtab_users[tab_cls];
        }
    }
    auto drop_table_use = [&]() {
        if (!tab_sp) return;
        std::lock_guard<std::mutex> lock(g_mu);
        --tab_sp->mtab_users[tab_cls];
    };
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        drop_table_use();
        return hip_fail(hipGetLastError(), "graph capture stream");
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        t_capturing = true;
        rc = transform(true, false, L, spin, batch, sampling, precision, flm_in, map, workspace, ws_bytes, cs);
        if (rc == SHT_OK)
            rc = transform(false, false, L, spin, batch, sampling, precision, map, flm_out, workspace, ws_bytes, cs);
        t_capturing = false;
        e = hipStreamEndCapture(cs, &g);  // always ends the capture
        if (rc == SHT_OK && e != hipSuccess) {
            rc = hip_fail(e, "graph end capture");
        }
    } else {
        rc = hip_fail(e, "graph begin capture");
    }
    hipGraphExec_t ex = nullptr;
    if (rc == SHT_OK) {
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            rc = hip_fail(e, "graph instantiate");
        }
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc != SHT_OK) {
        drop_table_use();
        return rc;
    }
    sht_graph_s *h = new sht_graph_s{dev, ex, tab_sp, tab_cls};
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        g_graphs.insert(h);
    }
    *out = h;
    return SHT_OK;
}

int sht_graph_launch(sht_graph graph, void *stream) {
    hipGraphExec_t ex;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        if (!graph || !g_graphs.count(graph)) return SHT_ERR_INVALID_ARG;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev != graph->device) return SHT_ERR_INVALID_ARG;
        ex = graph->exec;
    }
    SHT_HIP(hipGraphLaunch(ex, (hipStream_t)stream), "graph launch");
    return SHT_OK;
}

int sht_graph_destroy(sht_graph graph) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (!graph || !g_graphs.count(graph)) return SHT_ERR_INVALID_ARG;
    g_graphs.erase(graph);
    const hipError_t e = hipGraphExecDestroy(graph->exec);
    if (graph->tab_sp) {
        std::lock_guard<std::mutex> lock(g_mu);
        --graph->tab_sp->mtab_users[graph->tab_cls];
    }
    delete graph;
    if (e != hipSuccess) return hip_fail(e, "graph destroy");
    return SHT_OK;
}

int sht_release_all(void) {
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (sht_graph_s *h : g_graphs) {
            (void)hipGraphExecDestroy(h->exec);
            delete h;
        }
        g_graphs.clear();
    }
    std::lock_guard<std::mutex> build(g_build_mu);  // no build runs meanwhile
    std::lock_guard<std::mutex> lock(g_mu);
    int rc = SHT_OK;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) cur = 0;
    for (auto &kv : g_spin) {
        (void)hipSetDevice(kv.second->device);
        if (hipFree(kv.second->wi - (size_t)kTabPad * kv.second->L) != hipSuccess) rc = SHT_ERR_HIP;
        if (kv.second->mtab64 && hipFree(kv.second->mtab64) != hipSuccess) rc = SHT_ERR_HIP;
        if (kv.second->mtab32 && hipFree(kv.second->mtab32) != hipSuccess) rc = SHT_ERR_HIP;
        delete kv.second;
    }
    g_spin.clear();
    for (auto &kv : g_plans) {
        (void)hipSetDevice(kv.second->device);
        if (hipFree(kv.second->f64.tw) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second->f32.tw) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second->rec.ri) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second->rec.rf) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second->rec.fab) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second->rec.jti - (size_t)kTabPad * kv.second->L) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second->rec.jtf - (size_t)kTabPad * kv.second->L) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second->rec.cl) != hipSuccess) rc = SHT_ERR_HIP;
        for (int md = 0; md < 2; ++md)
            for (int c = 0; c < 2; ++c)
                if (kv.second->rec.sched[md][c] && hipFree(kv.second->rec.sched[md][c]) != hipSuccess) rc = SHT_ERR_HIP;
        delete kv.second;
    }
    g_plans.clear();
    for (auto &kv : g_devices) {
        (void)hipSetDevice(kv.first);
        if (hipFree(kv.second.E.mant) != hipSuccess) rc = SHT_ERR_HIP;
        if (hipFree(kv.second.E.expo) != hipSuccess) rc = SHT_ERR_HIP;
    }
    g_devices.clear();
    for (auto &kv : g_build_streams) {
        (void)hipSetDevice(kv.first);
        if (hipStreamDestroy(kv.second) != hipSuccess) rc = SHT_ERR_HIP;
    }
    g_build_streams.clear();
    (void)hipSetDevice(cur);
    return rc;
}

const char *sht_status_string(int status) {
    switch (status) {
        case SHT_OK: return "ok";
        case SHT_ERR_INVALID_ARG: return "invalid argument (L, spin, batch or a NULL pointer)";
        case SHT_ERR_UNSUPPORTED: return "unsupported sampling or precision";
        case SHT_ERR_WORKSPACE: return "workspace smaller than sht_workspace_bytes()";
        case SHT_ERR_ALIGNMENT: return "misaligned buffer";
        case SHT_ERR_OOM: return "device allocation for a plan failed";
        case SHT_ERR_HIP: return "HIP error (see sht_last_hip_error)";
        case SHT_ERR_BUSY: return "resource in use (a captured graph streams this table)";
        case SHT_ERR_NOT_READY: return "plan not resident (call sht_plan_warmup first)";
        default: return "unknown status";
    }
}

int sht_version(void) { return SHT_VERSION; }

const char *sht_last_hip_error(void) { return g_last_hip_error; }

int sht_trace_enable(int on) {
    g_trace_on = on != 0;
    return SHT_OK;
}

int sht_trace_read(double *ms, int *count, int nstages) {
    if ((!ms || !count) && nstages > 0) return SHT_ERR_INVALID_ARG;
    std::vector<TraceRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_trace_mu);
        recs.swap(g_trace_pending);
    }
    int rc = SHT_OK;
    for (const TraceRec &r : recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            rc = hip_fail(hipGetLastError(), "trace read");
        } else if (r.stage < nstages) {
            ms[r.stage] += (double)t;
            count[r.stage] += 1;
        }
    }
    std::lock_guard<std::mutex> lk(g_trace_mu);
    for (const TraceRec &r : recs) {
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    return rc;
}

}  // extern "C"
