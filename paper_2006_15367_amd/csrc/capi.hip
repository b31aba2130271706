// C ABI of the MLFMA library: handles, uploads, and the order of the
// kernels of one matvec (paper Sec. 2 five-stage list: C2M, M2M, M2L, L2L,
// L2O, plus the leaf-level near field).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace mlfma {
const char *last_error_text();
}

using namespace mlfma;

namespace {

std::atomic<int64_t> g_mem_limit{0};

// interpolation / anterpolation variant value of the fused pair kernel
constexpr int kPairVariant = 4;

struct DevLevel {
    int64_t nbox = 0;
    int L = 0, nth = 0, nph = 0;
    int64_t K = 0;
    int ntypes = 0;
    float4 *khat_w = nullptr;
    float2 *T = nullptr;
    // sampled operators (MLFMA_SAMPLED_OPERATORS): tables [nrad][Msamp + 1]
    // against the angle to the offset, unit offsets with their table row
    float2 *Tsamp = nullptr;
    float4 *xr = nullptr;
    double *trig64 = nullptr;        // (cos, sin) of the theta nodes, then of phi
    int Msamp = 0;
    int32_t *far_start = nullptr, *far_src = nullptr;
    int16_t *far_type = nullptr;
    int64_t n_far = 0;
    int32_t *parent = nullptr;       // into level-1
    uint8_t *oct = nullptr;          // octant of the box inside its parent
    int32_t *child_start = nullptr;  // into level+1
    int32_t *nbr_start = nullptr, *nbr_idx = nullptr;  // neighbours at this level
    int32_t *base = nullptr;         // 49 cx + 7 cy + cz
    int16_t *typemap = nullptr;      // [343] offset code -> operator or -1
    int m2l_variant = 0;             // 0 per-observer (L2), 1 operators in LDS, 2 sibling groups,
                                     // 3 sibling groups with per-source records, 4 = 3 with
                                     // the slice-major sweep, 5 = 3 record-balanced, 6 = 5 on
                                     // 32-sample slices, 7 = 5 on antipodal slices, 8 = 5 on
                                     // octant slices, 9 = 3 on the matrix cores (several RHS)
    float m2l_alone[10] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1};  // autotuner, ms per form
    int32_t *rec_start = nullptr, *rec_src = nullptr;  // records of the parents (level l-1)
    int32_t *rec_off = nullptr;      // [records][8] LDS byte offsets of the operators
    // antipodal slices (one-RHS variant 7): operators of one offset of each
    // +-pair in slice-lane order [ntp][Kp], slice lane -> sample [Kp], and
    // the record slots as pair * 512 | (negated ? 504 : 0)
    float2 *Tp = nullptr;
    int32_t *aperm = nullptr, *rec_off_anti = nullptr;
    int ntp = 0;
    int64_t Kp = 0;
    // octant slices (one-RHS variant 8): operators of the offsets
    // (|dx|, |dy|, |dz|) in slice-lane order [nto][Ko], slot codes [Ko]
    // (sample, or -(sample + 2) for a repeated direction, -1 padding), and
    // the record slots as row * 512 | 8 g (g: reflections x, y, z as bits
    // 2, 1, 0)
    float2 *To = nullptr;
    int32_t *operm = nullptr, *rec_off_oct = nullptr;
    int nto = 0;
    int64_t Ko = 0;
    float2 *S = nullptr, *Lloc = nullptr;  // [nbox][R][K]
    int Lc = 0, Mc = 0;
    float2 *shift = nullptr, *shift_axis = nullptr;
    float *iF = nullptr, *iA = nullptr, *iG = nullptr;
    float *aF = nullptr, *aB = nullptr, *aG = nullptr;
    // level pair (this level = parent): 0 three passes through HBM, 1 + k
    // one pass in work split k, 4 the fused pair kernel
    int interp_variant = 0, anterp_variant = 0;
    // autotuner: ms alone of each of those variants (negative: not timed)
    float interp_alone[5] = {-1, -1, -1, -1, -1}, anterp_alone[5] = {-1, -1, -1, -1, -1};
    bool onepass_ok = false;         // the one-pass kernels fit in LDS
    // fused pair kernel: parent groups (first, one past last) and operator
    // fragment tables of each direction
    bool pair_ok[2] = {false, false};
    int4 *ptile[2] = {nullptr, nullptr};
    int64_t nptile[2] = {0, 0};
    float *pfr[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
};

}  // namespace

struct mlfma_ops_s {
    Tree *tree = nullptr;
    double k = 0;
    int digits = 0, max_rhs = 0;
    uint32_t flags = 0;
    int device = 0;
    int64_t n = 0;
    int n_lev = 0;
    std::vector<LevelTables> tab;  // host tables (kept for info queries)
    std::vector<DevLevel> lev;
    float4 *pts = nullptr;
    int32_t *perm = nullptr, *pt_leaf = nullptr, *pt_start = nullptr;
    int32_t *near_start = nullptr, *near_idx = nullptr, *leaf_coord = nullptr;
    int2 *p2p_items = nullptr;       // (leaf, first target) per 64-target chunk
    int64_t n_p2p_items = 0, n_p2p_heavy = 0;
    float2 *qs = nullptr, *near = nullptr;
    float2 *fq = nullptr, *fg = nullptr;  // fields for the position gradient [n][R][3]
    float2 *X1 = nullptr, *X2 = nullptr;
    int64_t scratch_elems = 0;
    uint64_t pos_version = 0;
    std::vector<void *> allocs;
    int64_t last_R = 0;
    // library streams for the concurrent schedule (near field; M2L) and
    // the events that fork and join them
    hipStream_t side[2] = {nullptr, nullptr};
    // concurrent: where the near field forks: 0 start of the downward pass,
    // 1 start of the matvec, 2 after C2M, 3 / 4 after the first / second M2M
    // of the upward pass
    int near_fork = 0;
    // concurrent: eighths of the CUs the M2L workgroups of levels > 3 may
    // hold (timed at precompute with the fork point)
    int m2l_share8 = 6;
    // concurrent: 1 = the leaf level's M2L runs after the coarser levels'
    // on its stream, during the downward pass (it is first needed by the
    // last L2L), instead of beside the upward pass
    int leaf_late = 0;
    // concurrent, fork after an M2M: 1 = the near field in two halves of its
    // work items, the second forked after the next M2M
    int near_split = 0;
    // GMRES workspace: Krylov basis [(gm_cap + 1) x n], work vector,
    // dot-product partials, coefficient vector (allocated on first solve)
    int gm_cap = 0;
    float2 *gm_V = nullptr, *gm_w = nullptr;
    double2 *gm_part = nullptr, *gm_c = nullptr;
    int64_t planned_bytes = 0;       // device bytes of the precompute
    int64_t operator_bytes = 0;      // of which translation operators
    bool sampled = false;            // MLFMA_SAMPLED_OPERATORS
    hipEvent_t ev_fork = nullptr, ev_near = nullptr, ev_m2l = nullptr, ev_leaf = nullptr;
    std::vector<hipEvent_t> ev_S;  // per level: multipoles ready
    // captured graphs of previous calls (MLFMA_USE_GRAPH)
    struct GraphEntry {
        const void *q = nullptr;
        void *out = nullptr;
        int64_t nrhs = 0;
        int dtype = 0, field = 0, cin = 0, cout = 0, odt = 0;
        uint32_t parts = 0;
        hipStream_t stream = nullptr;
        hipGraphExec_t exec = nullptr;
        uint64_t use = 0;
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    // launch timing (diagnostics).  prof_ev is a pool: a session uses its
    // first 2 prof_cap events; up to kProfPoolKeep of them outlive the
    // session, so that a session of the same size started inside a timed
    // loop creates no events there
    uint32_t prof_mask = 0;
    int64_t prof_cap = 0, prof_used = 0;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_id;
};

constexpr size_t kProfPoolKeep = 8192;

#define CK(x)                                                   \
    do {                                                        \
        hipError_t _e = (x);                                    \
        if (_e != hipSuccess) return check_hip(_e, #x);         \
    } while (0)

// launch `x` (a dev:: launcher) as kernel `id`, bracketed by profiling
// events when that id is being timed
#define LAUNCH(id, x)                                           \
    do {                                                        \
        const int _p = prof_start(o, (id), s);                  \
        hipError_t _e = (x);                                    \
        if (_p) prof_stop(o, s, _p);                            \
        if (_e != hipSuccess) return check_hip(_e, #x);         \
    } while (0)

namespace {

// ---------------------------------------------------------------- memory --
struct Planner {
    int64_t bytes = 0;
    void add(int64_t b) { bytes += (b + 255) / 256 * 256; }
};

// Timing of one launcher call: 0 not timed; 1 event markers recorded on
// the stream before and after the call; 2 (M2L) events handed to the
// launch itself (dev::launch_timing), which records the kernel's own start
// and end and adds nothing to the stream between kernels.
int prof_start(mlfma_ops_s *o, int id, hipStream_t s)
{
    if (!(o->prof_mask & (1u << id)) || o->prof_used >= o->prof_cap) return 0;
    o->prof_id[o->prof_used] = id;
    if (id == MLFMA_K_M2L) {
        dev::launch_timing.start = o->prof_ev[2 * o->prof_used];
        dev::launch_timing.stop = o->prof_ev[2 * o->prof_used + 1];
        dev::launch_timing.used = false;
        return 2;
    }
    if (hipEventRecord(o->prof_ev[2 * o->prof_used], s) != hipSuccess) return 0;
    return 1;
}

void prof_stop(mlfma_ops_s *o, hipStream_t s, int mode)
{
    if (mode == 2) {
        const bool used = dev::launch_timing.used;  // false: nothing was launched
        dev::launch_timing = dev::LaunchTiming();
        if (used) ++o->prof_used;
        return;
    }
    (void)hipEventRecord(o->prof_ev[2 * o->prof_used + 1], s);
    ++o->prof_used;
}

// End a session; keep at most `keep` pooled events (0: destroy them all)
void prof_release(mlfma_ops_s *o, size_t keep = 0)
{
    if (o->prof_ev.size() > keep) {
        for (hipEvent_t e : o->prof_ev) (void)hipEventDestroy(e);
        o->prof_ev.clear();
    }
    o->prof_id.clear();
    o->prof_mask = 0;
    o->prof_cap = o->prof_used = 0;
}

template <typename T>
int dalloc(mlfma_ops_s *o, T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) return MLFMA_OK;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? MLFMA_ENOMEM : MLFMA_EDEVICE,
                    "hipMalloc(%lld bytes): %s", (long long)(count * sizeof(T)),
                    hipGetErrorString(e));
    }
    o->allocs.push_back(q);
    *p = (T *)q;
    return MLFMA_OK;
}

template <typename T>
int upload(mlfma_ops_s *o, T **p, const T *src, int64_t count)
{
    int rc = dalloc(o, p, count);
    if (rc || count <= 0) return rc;
    hipError_t e = hipMemcpy(*p, src, (size_t)count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(MLFMA_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    return MLFMA_OK;
}

void free_graphs(mlfma_ops_s *o)
{
    for (auto &g : o->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    o->graphs.clear();
}

void free_ops(mlfma_ops_s *o)
{
    if (!o) return;
    prof_release(o);
    free_graphs(o);
    {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess) {
            (void)hipSetDevice(o->device);
            for (hipStream_t &st : o->side)
                if (st) (void)hipStreamDestroy(st);
            for (hipEvent_t e : {o->ev_fork, o->ev_near, o->ev_m2l, o->ev_leaf})
                if (e) (void)hipEventDestroy(e);
            for (hipEvent_t e : o->ev_S)
                if (e) (void)hipEventDestroy(e);
            (void)hipSetDevice(cur);
        }
    }
    if (!o->allocs.empty()) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess) {
            (void)hipSetDevice(o->device);
            for (void *p : o->allocs) (void)hipFree(p);
            (void)hipSetDevice(cur);
        }
    }
    release_tree(o->tree);
    delete o;
}

// leaf-local FP32 offsets of the sorted points
std::vector<float4> point_offsets(const Tree &t)
{
    std::vector<float4> p(t.n);
    const HostLevel &leaf = t.lev[t.n_lev];
    for (int64_t s = 0; s < t.n; ++s) {
        const int64_t i = t.perm[s];
        const int32_t *c = &leaf.coord[3 * t.pt_leaf[s]];
        float v[3];
        for (int a = 0; a < 3; ++a) {
            const double centre = t.origin[a] + (c[a] + 0.5) * t.leaf;
            v[a] = (float)(t.xyz[3 * i + a] - centre);
        }
        p[s] = make_float4(v[0], v[1], v[2], 0.f);
    }
    return p;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return MLFMA_OK;
    return fail(MLFMA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int refresh_positions(mlfma_ops_s *o)
{
    if (o->pos_version == o->tree->pos_version) return MLFMA_OK;
    std::vector<float4> p = point_offsets(*o->tree);
    // calls still running on other streams (the caller's, the library's
    // side streams) read the positions: let them finish before the upload
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return check_hip(e, "position upload: device synchronize");
    e = hipMemcpy(o->pts, p.data(), p.size() * sizeof(float4), hipMemcpyHostToDevice);
    if (e != hipSuccess) return check_hip(e, "position upload");
    o->pos_version = o->tree->pos_version;
    return MLFMA_OK;
}

// M2L forms that run on sampled operators (the record kernels that stage
// the operator slice themselves)
bool sampled_m2l_form(int v) { return (v >= 3 && v <= 5) || v == 9; }

// ---------------------------------------------------------------- matvec --
// max_wg: workgroup cap of the record variants (0: one per CU)
hipError_t launch_m2l(mlfma_ops_s *o, int l, int variant, int R, hipStream_t s, int max_wg = 0)
{
    DevLevel &D = o->lev[l];
    DevLevel &Pl = o->lev[l - 1];
    if (o->sampled) {
        // record kernels with the operator slice interpolated from the tables
        if (!sampled_m2l_form(variant)) return hipErrorInvalidValue;
        dev::SampledT st;
        st.tab = D.Tsamp;
        st.xr = D.xr;
        st.trig = D.trig64;
        st.nth = D.nth;
        st.nph = D.nph;
        st.M = D.Msamp;
        if (variant == 9)
            return dev::m2l_mfma(Pl.nbox, D.K, D.ntypes, Pl.child_start, D.rec_start, D.rec_src,
                                 D.rec_off, nullptr, D.S, R, D.Lloc, s, max_wg, st);
        return dev::m2l_rec(Pl.nbox, D.K, D.ntypes, Pl.child_start, D.rec_start, D.rec_src,
                            D.rec_off, nullptr, D.S, R, D.Lloc, s, variant - 3, max_wg, st);
    }
    switch (variant) {
    case 9:
        return dev::m2l_mfma(Pl.nbox, D.K, D.ntypes, Pl.child_start, D.rec_start, D.rec_src,
                             D.rec_off, D.T, D.S, R, D.Lloc, s, max_wg);
    case 1:
        return dev::m2l_lds(D.nbox, D.K, D.ntypes, D.far_start, D.far_src, D.far_type, D.T, D.S,
                            R, D.Lloc, s);
    case 2:
        return dev::m2l_sg(Pl.nbox, D.K, D.ntypes, Pl.child_start, Pl.nbr_start, Pl.nbr_idx,
                           D.base, D.typemap, D.T, D.S, R, D.Lloc, s);
    case 7:
        if (R == 1)
            return dev::m2l_anti(Pl.nbox, D.K, D.ntp, Pl.child_start, D.rec_start, D.rec_src,
                                 D.rec_off_anti, D.Tp, D.aperm, D.Kp, D.S, D.Lloc, s, max_wg);
        return dev::m2l_rec(Pl.nbox, D.K, D.ntypes, Pl.child_start, D.rec_start, D.rec_src,
                            D.rec_off, D.T, D.S, R, D.Lloc, s, 2, max_wg);
    case 8:
        if (R == 1)
            return dev::m2l_anti(Pl.nbox, D.K, D.nto, Pl.child_start, D.rec_start, D.rec_src,
                                 D.rec_off_oct, D.To, D.operm, D.Ko, D.S, D.Lloc, s, max_wg, 8);
        return dev::m2l_rec(Pl.nbox, D.K, D.ntypes, Pl.child_start, D.rec_start, D.rec_src,
                            D.rec_off, D.T, D.S, R, D.Lloc, s, 2, max_wg);
    case 3:
    case 4:
    case 5:
    case 6:
        return dev::m2l_rec(Pl.nbox, D.K, D.ntypes, Pl.child_start, D.rec_start, D.rec_src,
                            D.rec_off, D.T, D.S, R, D.Lloc, s, variant - 3, max_wg);
    default:
        return dev::m2l(D.nbox, D.K, D.far_start, D.far_src, D.far_type, D.T, D.S, R, D.Lloc, s);
    }
}

// Fused pair kernel of the level pair (l, l+1): M2M (down = 0) or L2L.
hipError_t launch_pair(mlfma_ops_s *o, int l, int R, hipStream_t s, int down)
{
    DevLevel &P = o->lev[l], &C = o->lev[l + 1];
    return dev::pair_map(C.L, P.L, down != 0, down ? P.Lloc : C.S, down ? C.Lloc : P.S,
                         P.ptile[down], P.nptile[down], R, P.pfr[down][0], P.pfr[down][1],
                         P.pfr[down][2], P.shift_axis, P.shift, s,
                         (o->flags & MLFMA_BF16X3_INTERP) != 0);
}

// One-pass interpolation / anterpolation of the level pair (l, l+1).
hipError_t launch_interp_onepass(mlfma_ops_s *o, int l, int R, hipStream_t s, int shape)
{
    DevLevel &P = o->lev[l], &C = o->lev[l + 1];
    return dev::interp_fused(P.nbox, R, C.L, P.L, shape, P.child_start, C.oct, C.S, P.iF, P.iA,
                             P.iG, P.shift_axis, P.S, s);
}

hipError_t launch_anterp_onepass(mlfma_ops_s *o, int l, int R, hipStream_t s, int shape)
{
    DevLevel &P = o->lev[l], &C = o->lev[l + 1];
    return dev::anterp_fused(P.nbox, R, C.L, P.L, shape, P.child_start, C.oct, P.Lloc, P.aF,
                             P.aB, P.aG, P.shift_axis, C.Lloc, s);
}

// Three-pass interpolation / anterpolation of the level pair (l, l+1).
hipError_t launch_interp_staged(mlfma_ops_s *o, int l, int R, hipStream_t s)
{
    DevLevel &P = o->lev[l], &C = o->lev[l + 1];
    const bool b3 = (o->flags & MLFMA_BF16X3_INTERP) != 0;
    hipError_t e = dev::interp_s1(C.S, C.nbox * R, C.nth, C.nph, P.iF, P.Mc, o->X1, s, b3);
    if (e == hipSuccess)
        e = dev::theta_map(o->X1, C.nbox * R, C.nth, P.Mc, P.iA, P.nth, o->X2, s, b3);
    if (e == hipSuccess)
        e = dev::interp_s3(P.nbox, R, P.nth, P.nph, P.Mc, P.child_start, C.oct, o->X2, P.iG,
                           P.shift, P.S, s);
    return e;
}

hipError_t launch_anterp_staged(mlfma_ops_s *o, int l, int R, hipStream_t s)
{
    DevLevel &P = o->lev[l], &C = o->lev[l + 1];
    const bool b3 = (o->flags & MLFMA_BF16X3_INTERP) != 0;
    hipError_t e = dev::anterp_s1(P.Lloc, C.parent, C.oct, C.nbox, R, P.nth, P.nph, P.shift,
                                  P.aF, P.Mc, o->X1, s, b3);
    if (e == hipSuccess)
        e = dev::theta_map(o->X1, C.nbox * R, P.nth, P.Mc, P.aB, C.nth, o->X2, s, b3);
    if (e == hipSuccess)
        e = dev::anterp_s3(C.nbox, R, C.nth, C.nph, P.Mc, o->X2, P.aG, C.Lloc, s, b3);
    return e;
}

// Best of 3 HIP-event timings of one launch sequence; negative on failure.
template <class F>
float time_best(hipStream_t s, hipEvent_t e0, hipEvent_t e1, F &&run)
{
    float tmin = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, s);
        const hipError_t e = run();
        (void)hipEventRecord(e1, s);
        if (e != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.f;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        tmin = std::min(tmin, ms);
    }
    return tmin;
}

// Autotuner: per level, time every M2L variant and, per level pair, the
// one-pass and three-pass interpolation and anterpolation (HIP events,
// best of 3) at the handle's max_rhs, and keep the fastest.  The variants
// compute the same result up to summation order.
int autotune(mlfma_ops_s *o)
{
    if (o->n_lev < 3) return MLFMA_OK;
    hipStream_t s;
    if (hipStreamCreate(&s) != hipSuccess) return fail(MLFMA_EDEVICE, "autotune: stream");
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int R = o->max_rhs;
    int rc = MLFMA_OK;
    for (int l = 3; l <= o->n_lev && rc == MLFMA_OK; ++l) {
        float best = 1e30f;
        int bestv = 0;
        for (int v = 0; v < 10; ++v) {
            if (v >= 6 && v <= 8 && R != 1) continue;  // variants 6, 7 and 8 serve one RHS
            if (v == 9 && R == 1) continue;  // the matrix-core form needs several RHS
            if (o->sampled && !sampled_m2l_form(v)) continue;
            const float t = time_best(s, e0, e1, [&] { return launch_m2l(o, l, v, R, s); });
            if (t < 0.f) {
                rc = fail(MLFMA_EDEVICE, "autotune: M2L variant %d failed", v);
                break;
            }
            o->lev[l].m2l_alone[v] = t;
            if (t < best) {
                best = t;
                bestv = v;
            }
        }
        o->lev[l].m2l_variant = bestv;
    }
    const bool b3 = (o->flags & MLFMA_BF16X3_INTERP) != 0;
    for (int l = 3; l < o->n_lev && rc == MLFMA_OK; ++l) {
        DevLevel &P = o->lev[l];
        // (BF16x3: the three passes and the pair kernel; the one-pass
        // kernels are FP32 only)
        if (!((P.onepass_ok && !b3) || P.pair_ok[0] || P.pair_ok[1])) continue;
        // variant 0: three passes; 1 + k: one pass in work split k
        float bi = time_best(s, e0, e1, [&] { return launch_interp_staged(o, l, R, s); });
        float ba = time_best(s, e0, e1, [&] { return launch_anterp_staged(o, l, R, s); });
        if (bi < 0.f || ba < 0.f) {
            rc = fail(MLFMA_EDEVICE, "autotune: interpolation variants failed on level %d", l);
            break;
        }
        P.interp_variant = P.anterp_variant = 0;
        P.interp_alone[0] = bi;
        P.anterp_alone[0] = ba;
        for (int dn = 0; dn < 2 && rc == MLFMA_OK; ++dn) {
            if (!P.pair_ok[dn]) continue;
            const float tp = time_best(s, e0, e1, [&] { return launch_pair(o, l, R, s, dn); });
            if (tp < 0.f) {
                rc = fail(MLFMA_EDEVICE, "autotune: pair kernel failed on level %d", l);
                break;
            }
            (dn ? P.anterp_alone : P.interp_alone)[kPairVariant] = tp;
            float &best = dn ? ba : bi;
            if (tp < best) {
                best = tp;
                (dn ? P.anterp_variant : P.interp_variant) = kPairVariant;
            }
        }
        if (rc != MLFMA_OK) break;
        const int nsh = (P.onepass_ok && !b3) ? dev::pair_onepass_shapes(o->lev[l + 1].L, P.L) : 0;
        for (int k = 0; k < nsh && rc == MLFMA_OK; ++k) {
            const float tf = time_best(s, e0, e1, [&] { return launch_interp_onepass(o, l, R, s, k); });
            const float af = time_best(s, e0, e1, [&] { return launch_anterp_onepass(o, l, R, s, k); });
            if (tf < 0.f || af < 0.f) {
                rc = fail(MLFMA_EDEVICE, "autotune: one-pass variant %d failed on level %d", k, l);
                break;
            }
            P.interp_alone[1 + k] = tf;
            P.anterp_alone[1 + k] = af;
            if (tf < bi) {
                bi = tf;
                P.interp_variant = 1 + k;
            }
            if (af < ba) {
                ba = af;
                P.anterp_variant = 1 + k;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return rc;
}

// The far field: C2M, M2M up the tree, M2L per level, L2L down the tree.
// Leaves the leaf-level local expansions in lev[n_lev].Lloc.  With `conc`
// the M2L of a level runs on library stream side[1] as soon as the level's
// multipoles are ready (event), overlapping the rest of the M2M chain; the
// L2L chain waits for the last M2L.
template <class Near>
int run_far(mlfma_ops_s *o, int R, hipStream_t s, bool conc, Near &&near)
{
    const int fork = conc ? o->near_fork : 1;
    const int nl = o->n_lev;
    DevLevel &leaf = o->lev[nl];
    const float kw = (float)o->k;
    const bool b3 = (o->flags & MLFMA_BF16X3_INTERP) != 0;
    hipStream_t sm = conc ? o->side[1] : s;
    bool side_used = false;  // an M2L ran on sm
    auto m2l_level = [&](int l) -> int {
        // level 3, the last, stays on the caller's stream: the downward
        // pass waits for it anyway, and a fork and join around it cost
        // more than the overlap gains
        const bool side = conc && l > 3;
        if (side) {
            side_used = true;
            CK(hipEventRecord(o->ev_S[l], s));
            CK(hipStreamWaitEvent(sm, o->ev_S[l], 0));
        }
        hipStream_t s0 = s;
        hipStream_t s = side ? sm : s0;
        DevLevel &D = o->lev[l];
        // concurrent: the record variants take m2l_share8 / 8 of the CUs
        // (their workgroups hold much or all of a CU's LDS) and leave the
        // rest to the upward chain, the critical path, which otherwise
        // waits for M2L workgroups to retire
        const int cap = side ? dev::cu_count() * o->m2l_share8 / 8 : 0;
        LAUNCH(MLFMA_K_M2L, launch_m2l(o, l, D.m2l_variant, R, s, cap));
        return MLFMA_OK;
    };
    LAUNCH(MLFMA_K_C2M, dev::c2m(o->pts, o->pt_start, leaf.nbox, leaf.khat_w, leaf.K, kw, o->qs, R, leaf.S, s));
    bool near_done = false;
    if (fork == 2) {
        if (int r = near(nullptr, 0)) return r;
        near_done = true;
    }
    const bool split = conc && o->near_split && fork >= 3;
    bool split_pending = false;
    // leaf M2L late: it is enqueued on the M2L stream after the coarser
    // levels' M2L, whose forks (recorded here on s after C2M and the M2Ms)
    // already order it after C2M; only a four-level tree, whose one
    // coarser level runs on s, needs an event of its own (a marker on s
    // costs about 5 us of the critical path)
    const bool leaf_late = conc && o->leaf_late && nl > 3;
    const bool leaf_event = leaf_late && nl == 4;
    if (leaf_event)
        CK(hipEventRecord(o->ev_S[nl], s));
    else if (!leaf_late)
        if (int r = m2l_level(nl)) return r;
    for (int l = nl - 1; l >= 3; --l) {
        DevLevel &P = o->lev[l], &C = o->lev[l + 1];
        const int M = P.Mc;
        if (P.interp_variant == kPairVariant) {
            LAUNCH(MLFMA_K_INTERP, launch_pair(o, l, R, s, 0));
        } else if (P.interp_variant >= 1) {
            LAUNCH(MLFMA_K_INTERP, launch_interp_onepass(o, l, R, s, P.interp_variant - 1));
        } else {
            LAUNCH(MLFMA_K_INTERP_S1, dev::interp_s1(C.S, C.nbox * R, C.nth, C.nph, P.iF, M, o->X1, s, b3));
            LAUNCH(MLFMA_K_INTERP_S2, dev::theta_map(o->X1, C.nbox * R, C.nth, M, P.iA, P.nth, o->X2, s, b3));
            LAUNCH(MLFMA_K_INTERP_S3, dev::interp_s3(P.nbox, R, P.nth, P.nph, M, P.child_start, C.oct, o->X2, P.iG,
                              P.shift, P.S, s));
        }
        if (int r = m2l_level(l)) return r;
        // fork points 3 and 4: after the first or second M2M of the upward
        // pass (C2M and the finest M2Ms then run without the near field);
        // the near-field stream waits on the event the M2L fork of this
        // level recorded at the same point (one marker fewer)
        if (!near_done && ((fork == 3 && l == nl - 1) || (fork == 4 && l == nl - 2))) {
            if (int r = near(conc && l > 3 ? o->ev_S[l] : nullptr, split ? 1 : 0)) return r;
            near_done = true;
            split_pending = split;
        } else if (split_pending) {
            // the second half after the next M2M
            if (int r = near(conc && l > 3 ? o->ev_S[l] : nullptr, 2)) return r;
            split_pending = false;
        }
    }
    if (split_pending)
        if (int r = near(nullptr, 2)) return r;
    // the near field forked here fills the device during the downward
    // pass, whose small kernels leave most CUs idle (forked at the start,
    // it takes CUs from C2M and the upward chain)
    if (fork == 0 || (fork >= 3 && !near_done))
        if (int r = near(nullptr, 0)) return r;
    // join the M2L stream: an event recorded on it is part of a captured
    // graph only once it waited on an event of the capture, so where no
    // coarser level ran on it (four levels, leaf late) it first takes the
    // leaf M2L's wait, and where no M2L ran on it at all there is no join
    if (leaf_event) CK(hipStreamWaitEvent(sm, o->ev_S[nl], 0));
    if (conc && (side_used || leaf_late)) {
        CK(hipEventRecord(o->ev_m2l, sm));
        if (leaf_late) {
            hipStream_t s = sm;  // (LAUNCH times on the launch stream)
            const int cap = dev::cu_count() * o->m2l_share8 / 8;
            LAUNCH(MLFMA_K_M2L, launch_m2l(o, nl, leaf.m2l_variant, R, s, cap));
            CK(hipEventRecord(o->ev_leaf, s));
        }
        CK(hipStreamWaitEvent(s, o->ev_m2l, 0));
    }
    for (int l = 3; l < nl; ++l) {
        DevLevel &P = o->lev[l], &C = o->lev[l + 1];
        const int M = P.Mc;
        // the last L2L adds into the leaf locals the leaf M2L wrote
        if (leaf_late && l == nl - 1)
            CK(hipStreamWaitEvent(s, o->ev_leaf, 0));
        if (P.anterp_variant == kPairVariant) {
            LAUNCH(MLFMA_K_ANTERP, launch_pair(o, l, R, s, 1));
            continue;
        }
        if (P.anterp_variant >= 1) {
            LAUNCH(MLFMA_K_ANTERP, launch_anterp_onepass(o, l, R, s, P.anterp_variant - 1));
            continue;
        }
        LAUNCH(MLFMA_K_ANTERP_S1, dev::anterp_s1(P.Lloc, C.parent, C.oct, C.nbox, R, P.nth, P.nph, P.shift, P.aF, M,
                          o->X1, s, b3));
        LAUNCH(MLFMA_K_ANTERP_S2, dev::theta_map(o->X1, C.nbox * R, P.nth, M, P.aB, C.nth, o->X2, s, b3));
        LAUNCH(MLFMA_K_ANTERP_S3, dev::anterp_s3(C.nbox, R, C.nth, C.nph, M, o->X2, P.aG, C.Lloc, s, b3));
    }
    return MLFMA_OK;
}

// The near field and the far field from the gathered charges o->qs up to
// the leaf locals and o->near.  Concurrent schedule (side streams present,
// not disabled): the near field runs on side[0], forked at the start
// (o->near_fork 1), after C2M (2), after the first or second M2M (3, 4) or
// at the start of the downward pass (0),
// and joined on `s` at the end; the M2L of each level but the last (level
// 3) runs on side[1].
int run_core(mlfma_ops_s *o, int R, int field, uint32_t parts, hipStream_t s)
{
    const bool far = (parts & MLFMA_FAR) && o->n_lev >= 3;
    const int64_t nnear = o->n * R * (field ? 3 : 1);
    const bool conc = far && o->side[0] && !(o->flags & MLFMA_ONE_STREAM) &&
                      !(o->prof_mask & MLFMA_PROFILE_SERIAL);
    // `after`: an event already recorded on s at the fork point, or null
    // to record one; `part`: 0 all work items, 1 / 2 the first / second
    // half (the heavy items and half the others / the rest; the items
    // write disjoint targets)
    auto near = [&](hipEvent_t after, int part) -> int {
        if (conc) {
            if (!after) {
                CK(hipEventRecord(o->ev_fork, s));
                after = o->ev_fork;
            }
            CK(hipStreamWaitEvent(o->side[0], after, 0));
        }
        hipStream_t s0 = s;
        hipStream_t s = conc ? o->side[0] : s0;
        if (parts & MLFMA_NEAR) {
            int64_t i0 = 0, ni = o->n_p2p_items, nh = o->n_p2p_heavy;
            if (part) {
                const int64_t cut = o->n_p2p_heavy + (o->n_p2p_items - o->n_p2p_heavy) / 2;
                if (part == 1) {
                    ni = cut;
                } else {
                    i0 = cut;
                    ni = o->n_p2p_items - cut;
                    nh = 0;
                }
            }
            LAUNCH(MLFMA_K_P2P, dev::p2p(o->p2p_items + i0, ni, nh, o->pts,
                                         o->pt_start, o->near_start, o->near_idx, o->leaf_coord,
                                         (float)o->tree->leaf, (float)o->k, o->qs, R, field,
                                         o->near, s));
        } else if (part != 2) {
            LAUNCH(MLFMA_K_P2P, dev::zero(o->near, nnear, s));
        }
        if (conc) CK(hipEventRecord(o->ev_near, s));
        return MLFMA_OK;
    };
    auto none = [](hipEvent_t, int) -> int { return MLFMA_OK; };
    const bool early = !conc || o->near_fork == 1;
    if (early)
        if (int r = near(nullptr, 0)) return r;
    if (far) {
        const int r2 = early ? run_far(o, R, s, conc, none) : run_far(o, R, s, conc, near);
        if (r2) return r2;
    }
    if (conc) CK(hipStreamWaitEvent(s, o->ev_near, 0));
    return MLFMA_OK;
}

// Times the core (near + far field, max_rhs right-hand sides) on a scratch
// stream, as the concurrent schedule runs it, for the schedule tuners.
struct CoreTimer {
    mlfma_ops_s *o;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int reps = 3;
    bool warm = true;  // one untimed core before each timing
    explicit CoreTimer(mlfma_ops_s *o_) : o(o_) {}
    ~CoreTimer()
    {
        if (s) (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
    int init()
    {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return fail(MLFMA_EDEVICE, "schedule tuning: stream or event creation failed");
        // repetitions per timing: about 10 ms of cores (1 to 20), so that
        // short cores are timed above the run-to-run noise and long ones
        // (many RHS, 20-60 ms a core) do not make precompute slow; the
        // untimed core before each timing only for cores under 2 ms
        float t3 = 0.f;
        if (int r = time(&t3)) return r;  // three cores
        reps = std::max(1, std::min(20, (int)(30.f / std::max(t3, 1e-3f))));
        warm = t3 < 6.f;
        return MLFMA_OK;
    }
    // ms for `reps` cores after one untimed core
    int time(float *ms)
    {
        const int R = o->max_rhs;
        if (warm)
            if (int r = run_core(o, R, 0, MLFMA_NEAR | MLFMA_FAR, s)) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(MLFMA_EDEVICE, "schedule tuning: event");
        for (int rep = 0; rep < reps; ++rep)
            if (int r = run_core(o, R, 0, MLFMA_NEAR | MLFMA_FAR, s)) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return fail(MLFMA_EDEVICE, "schedule tuning: timing failed");
        return MLFMA_OK;
    }
};

// Pick where the concurrent schedule forks the near field and the share of
// the CUs the side-stream M2L may hold: time the core for each pair.
int tune_schedule(mlfma_ops_s *o)
{
    if (!o->side[0] || o->n_lev < 3) return MLFMA_OK;
    CoreTimer tm(o);
    if (int r = tm.init()) return r;
    float best = 1e30f;
    int best_cfg = 0;
    // M2L shares of 4/8 .. 8/8 of the CUs (8: uncapped) x the fork points
    // of the near field (3 and 4 where the upward pass has that many M2Ms)
    // x the leaf M2L early or late (trees of more than 3 levels); two
    // alternating rounds, best of the two per configuration
    constexpr int kShares[4] = {8, 7, 6, 4};
    const int nfork = std::min(5, 3 + std::max(0, o->n_lev - 3));
    const int nlate = o->n_lev > 3 ? 2 : 1;
    const int ncfg = 4 * nfork * nlate;
    auto apply = [&](int cfg) {
        o->near_fork = cfg % nfork;
        o->m2l_share8 = kShares[cfg / nfork % 4];
        o->leaf_late = cfg / (4 * nfork);
    };
    float t[40];
    for (float &x : t) x = 1e30f;
    for (int round = 0; round < 2; ++round)
        for (int cfg = 0; cfg < ncfg; ++cfg) {
            apply(cfg);
            float ms = 0.f;
            if (int r = tm.time(&ms)) return r;
            t[cfg] = std::min(t[cfg], ms);
        }
    for (int cfg = 0; cfg < ncfg; ++cfg)
        if (t[cfg] < best) {
            best = t[cfg];
            best_cfg = cfg;
        }
    apply(best_cfg);
    return MLFMA_OK;
}

// Refine the autotuner's per-kernel picks inside the concurrent schedule.
// Forms of one kernel whose times alone differ by a few percent need not
// rank the same way in the concurrent step, where they differ in the CUs
// and LDS they hold beside the upward chain and the near field (on the 262k
// sphere, one RHS, the leaf-adjacent M2L levels: the record form 5 and the
// octant form 8 within a few percent of each other alone, 2% apart in the
// step).  For each M2L level and each direction of each level pair, the
// variants within 25% of the fastest alone are timed in the whole core, in
// two alternating rounds, best of the two; a change needs a gain of 0.3%.
int refine_schedule(mlfma_ops_s *o)
{
    if (!o->side[0] || o->n_lev < 3) return MLFMA_OK;
    CoreTimer tm(o);
    if (int r = tm.init()) return r;
    // time each candidate value of `knob` (values below 10) in the core
    auto pick = [&](int &knob, const int *cand, int nc) -> int {
        if (nc < 2) return MLFMA_OK;
        const int cur = knob;
        float t[10];
        for (float &x : t) x = 1e30f;
        for (int round = 0; round < 2; ++round)
            for (int i = 0; i < nc; ++i) {
                knob = cand[i];
                float ms = 0.f;
                if (int r = tm.time(&ms)) {
                    knob = cur;
                    return r;
                }
                t[cand[i]] = std::min(t[cand[i]], ms);
            }
        int best = cur;
        for (int i = 0; i < nc; ++i)
            if (t[cand[i]] < t[best]) best = cand[i];
        knob = (t[cur] < 1e30f && t[best] >= 0.997f * t[cur]) ? cur : best;
        return MLFMA_OK;
    };
    auto refine = [&](int &knob, const float *alone, int nv) -> int {
        float fastest = 1e30f;
        for (int v = 0; v < nv; ++v)
            if (alone[v] >= 0.f) fastest = std::min(fastest, alone[v]);
        int cand[10], nc = 0;
        for (int v = 0; v < nv; ++v)
            if (alone[v] >= 0.f && alone[v] <= 1.25f * fastest) cand[nc++] = v;
        return pick(knob, cand, nc);
    };
    for (int l = o->n_lev; l >= 3; --l)
        if (int r = refine(o->lev[l].m2l_variant, o->lev[l].m2l_alone, 10)) return r;
    for (int l = o->n_lev - 1; l >= 3; --l) {
        DevLevel &P = o->lev[l];
        if (int r = refine(P.interp_variant, P.interp_alone, 5)) return r;
        if (int r = refine(P.anterp_variant, P.anterp_alone, 5)) return r;
    }
    if (o->near_fork >= 3) {
        const int halves[2] = {0, 1};
        if (int r = pick(o->near_split, halves, 2)) return r;
    }
    return MLFMA_OK;
}

// Schedule and kernel forms of the concurrent step: the schedule (fork
// point, CU share, leaf M2L order), then the forms inside it, then the
// schedule again for those forms, from two starting points: the forms
// fastest alone, and the octant M2L form (the least LDS per workgroup, so
// the most room for the kernels beside it) on every level but the leaf,
// with the record form on the leaf.
// The search is greedy and the step's optimum is joint: on the 262k sphere
// the second start reaches octant forms on levels 3..6 with the leaf's
// record form run late on half the CUs (0.557 ms), which no single change
// from the first start's result (0.571 ms) improves on.  The better of the
// two results, timed again in alternation, is kept.
int tune_concurrent(mlfma_ops_s *o)
{
    const int nl = o->n_lev;
    struct Pick {
        int fork, share, late, split;
        std::vector<int> m2l, interp, anterp;
    };
    auto save = [&]() {
        Pick p{o->near_fork, o->m2l_share8, o->leaf_late, o->near_split, {}, {}, {}};
        for (int l = 3; l <= nl; ++l) {
            p.m2l.push_back(o->lev[l].m2l_variant);
            p.interp.push_back(o->lev[l].interp_variant);
            p.anterp.push_back(o->lev[l].anterp_variant);
        }
        return p;
    };
    auto restore = [&](const Pick &p) {
        o->near_fork = p.fork;
        o->m2l_share8 = p.share;
        o->leaf_late = p.late;
        o->near_split = p.split;
        for (int l = 3; l <= nl; ++l) {
            o->lev[l].m2l_variant = p.m2l[l - 3];
            o->lev[l].interp_variant = p.interp[l - 3];
            o->lev[l].anterp_variant = p.anterp[l - 3];
        }
    };
    auto search = [&]() -> int {
        if (int r = tune_schedule(o)) return r;
        if (int r = refine_schedule(o)) return r;
        return tune_schedule(o);
    };
    const Pick start = save();
    if (int r = search()) return r;
    const Pick first = save();
    bool octant = false;
    restore(start);
    for (int l = 3; l < nl; ++l)
        if (o->lev[l].m2l_alone[8] >= 0.f && o->lev[l].m2l_variant != 8) {
            o->lev[l].m2l_variant = 8;
            octant = true;
        }
    if (!octant) {
        restore(first);
        return MLFMA_OK;
    }
    // and the leaf on the record form 5 (one workgroup per CU, the form
    // that leaves the most CUs whole to the kernels beside it when capped)
    if (o->lev[nl].m2l_alone[5] >= 0.f) o->lev[nl].m2l_variant = 5;
    if (int r = search()) return r;
    const Pick second = save();
    CoreTimer tm(o);
    if (int r = tm.init()) return r;
    float t1 = 1e30f, t2 = 1e30f;
    for (int round = 0; round < 3; ++round) {
        float ms = 0.f;
        restore(first);
        if (int r = tm.time(&ms)) return r;
        t1 = std::min(t1, ms);
        restore(second);
        if (int r = tm.time(&ms)) return r;
        t2 = std::min(t2, ms);
    }
    restore(t2 < t1 ? second : first);
    return MLFMA_OK;
}

// conj_in/conj_out: -1 = follow MLFMA_CONJ in parts
int do_matvec(mlfma_ops_s *o, const void *q, void *out, int64_t nrhs, int dtype,
              uint32_t parts, int field, hipStream_t s, int conj_in = -1, int conj_out = -1,
              int out_dtype = -1, bool allow_graph = true)
{
    if (!o) return fail(MLFMA_EINVAL, "matvec: ops handle is NULL");
    if (nrhs < 1 || nrhs > o->max_rhs)
        return fail(MLFMA_EINVAL, "matvec: nrhs=%lld outside 1..%d", (long long)nrhs, o->max_rhs);
    if (dtype != MLFMA_C64 && dtype != MLFMA_C128)
        return fail(MLFMA_EINVAL, "matvec: unknown dtype %d", dtype);
    if (!field && !(parts & (MLFMA_NEAR | MLFMA_FAR)))
        return fail(MLFMA_EINVAL, "matvec: parts must include MLFMA_NEAR or MLFMA_FAR");
    if (parts & ~7u) return fail(MLFMA_EINVAL, "matvec: unknown parts bits");
    if (field) parts = (parts & MLFMA_CONJ) | MLFMA_NEAR | MLFMA_FAR;
    if (o->n == 0) return MLFMA_OK;
    if (!q || !out) return fail(MLFMA_EINVAL, "matvec: null buffer");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(MLFMA_EDEVICE, "hipGetDevice failed");
    if (cur != o->device && hipSetDevice(o->device) != hipSuccess)
        return fail(MLFMA_EDEVICE, "hipSetDevice(%d) failed", o->device);
    int rc = refresh_positions(o);
    const int R = (int)nrhs;
    const int conj = (parts & MLFMA_CONJ) ? 1 : 0;
    const int cin = conj_in >= 0 ? conj_in : conj;
    const int cout = conj_out >= 0 ? conj_out : conj;
    const int odt = out_dtype >= 0 ? out_dtype : dtype;
    auto enqueue = [&]() -> int {
        const bool far = (parts & MLFMA_FAR) && o->n_lev >= 3;
        LAUNCH(MLFMA_K_GATHER, dev::gather(q, dtype, o->perm, o->n, R, cin, o->qs, s));
        if (int r = run_core(o, R, field, parts, s)) return r;
        DevLevel &leaf = o->lev[o->n_lev];
        if (far && !field && R >= 8) {
            // many right-hand sides: per-leaf product on the matrix cores
            LAUNCH(MLFMA_K_L2O, dev::l2o_leaf_mfma(o->pts, o->pt_start, leaf.nbox, o->perm,
                                                   leaf.khat_w, leaf.K, (float)o->k, leaf.Lloc,
                                                   o->near, R, cout, odt, out, s));
            return MLFMA_OK;
        }
        LAUNCH(MLFMA_K_L2O, dev::l2o_scatter(o->pts, o->pt_leaf, o->perm, far ? leaf.khat_w : nullptr,
                                             far ? leaf.K : 0, (float)o->k, far ? leaf.Lloc : nullptr,
                                             o->near, o->n, R, field, far ? 1 : 0, cout, odt, out, s));
        return MLFMA_OK;
    };
    const bool graph = rc == MLFMA_OK && allow_graph && (o->flags & MLFMA_USE_GRAPH) &&
                       s != nullptr && o->prof_mask == 0;
    if (rc == MLFMA_OK && !graph) rc = enqueue();
    if (rc == MLFMA_OK && graph) {
        mlfma_ops_s::GraphEntry *hit = nullptr;
        for (auto &g : o->graphs)
            if (g.q == q && g.out == out && g.nrhs == nrhs && g.dtype == dtype &&
                g.field == field && g.cin == cin && g.cout == cout && g.odt == odt &&
                g.parts == parts && g.stream == s)
                hit = &g;
        if (!hit) {
            hipGraph_t gph = nullptr;
            hipGraphExec_t exec = nullptr;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                (void)hipGetLastError();
                rc = fail(MLFMA_EDEVICE, "matvec: stream capture could not start");
            } else {
                const int rq = enqueue();
                const hipError_t ee = hipStreamEndCapture(s, &gph);
                if (rq) rc = rq;
                else if (ee != hipSuccess || !gph)
                    rc = fail(MLFMA_EDEVICE, "matvec: stream capture failed: %s", hipGetErrorString(ee));
                else if (hipGraphInstantiate(&exec, gph, nullptr, nullptr, 0) != hipSuccess)
                    rc = fail(MLFMA_EDEVICE, "matvec: graph instantiation failed");
                if (gph) (void)hipGraphDestroy(gph);
            }
            if (rc == MLFMA_OK) {
                if (o->graphs.size() >= 8) {
                    auto old = std::min_element(o->graphs.begin(), o->graphs.end(),
                                                [](const mlfma_ops_s::GraphEntry &a,
                                                   const mlfma_ops_s::GraphEntry &b) { return a.use < b.use; });
                    (void)hipGraphExecDestroy(old->exec);
                    o->graphs.erase(old);
                }
                mlfma_ops_s::GraphEntry ge;
                ge.q = q; ge.out = out; ge.nrhs = nrhs; ge.dtype = dtype; ge.field = field;
                ge.cin = cin; ge.cout = cout; ge.odt = odt; ge.parts = parts; ge.stream = s;
                ge.exec = exec;
                o->graphs.push_back(ge);
                hit = &o->graphs.back();
            }
        }
        if (rc == MLFMA_OK) {
            hit->use = ++o->graph_clock;
            rc = check_hip(hipGraphLaunch(hit->exec, s), "hipGraphLaunch");
        }
    }
    o->last_R = R;
    if (cur != o->device) (void)hipSetDevice(cur);
    return rc;
}

}  // namespace

// =================================================================== ABI ==
extern "C" {

int mlfma_build_tree(const double *xyz, int64_t n, double leaf_size, int max_levels, int device,
                     mlfma_tree_t *out)
{
    if (!out) return fail(MLFMA_EINVAL, "build_tree: out is NULL");
    Tree *t = nullptr;
    int rc = build_tree(xyz, n, leaf_size, max_levels, device, &t);
    if (rc) return rc;
    // mlfma_tree_s adds no members: reinterpret the Tree as the opaque handle
    *out = reinterpret_cast<mlfma_tree_t>(t);
    return MLFMA_OK;
}

int mlfma_update_positions(mlfma_tree_t t, const double *xyz)
{
    return update_positions(reinterpret_cast<Tree *>(t), xyz);
}

void mlfma_set_device_memory_limit(int64_t bytes) { g_mem_limit.store(bytes < 0 ? 0 : bytes); }

int mlfma_precompute_operators(mlfma_tree_t th, double k, int digits, int max_rhs,
                               uint32_t flags, mlfma_ops_t *out)
{
    if (!out) return fail(MLFMA_EINVAL, "precompute: out is NULL");
    *out = nullptr;
    Tree *t = reinterpret_cast<Tree *>(th);
    if (!t) return fail(MLFMA_EINVAL, "precompute: tree is NULL");
    if (!(k > 0.0) || !std::isfinite(k)) return fail(MLFMA_EINVAL, "precompute: k must be > 0");
    if (digits < 1 || digits > 10) return fail(MLFMA_EINVAL, "precompute: digits outside 1..10");
    if (max_rhs < 1 || max_rhs > 1024)
        return fail(MLFMA_EINVAL, "precompute: max_rhs outside 1..1024");
    if (flags & ~(uint32_t)(MLFMA_BF16X3_INTERP | MLFMA_NO_AUTOTUNE | MLFMA_USE_GRAPH |
                            MLFMA_ONE_STREAM | MLFMA_SAMPLED_OPERATORS))
        return fail(MLFMA_EINVAL, "precompute: unknown flags");
    // the near-field kernels evaluate exp(ikr) on the hardware sine/cosine,
    // whose argument (in turns, k r / 2 pi) must stay within +-256; near
    // pairs are at most 2 sqrt(3) leaf apart
    if (k * 2.0 * std::sqrt(3.0) * t->leaf / (2.0 * M_PI) > 250.0)
        return fail(MLFMA_EINVAL,
                    "precompute: leaf boxes of %g wavelengths exceed the near-field phase range "
                    "(at most about 72 wavelengths)",
                    k * t->leaf / (2.0 * M_PI));
    if (t->n_lev >= 3 && k * std::sqrt(3.0) * t->leaf < 1.0)
        return fail(MLFMA_EINVAL,
                    "precompute: leaf boxes too small for the diagonal form (k sqrt(3) a = %g < 1)",
                    k * std::sqrt(3.0) * t->leaf);

    mlfma_ops_s *o = new (std::nothrow) mlfma_ops_s();
    if (!o) return fail(MLFMA_ENOMEM, "precompute: out of host memory");
    o->tree = t;
    ++t->refcount;
    o->k = k;
    o->digits = digits;
    o->max_rhs = max_rhs;
    o->flags = flags;
    o->device = t->device;
    o->n = t->n;
    o->n_lev = t->n_lev;
    o->sampled = (flags & MLFMA_SAMPLED_OPERATORS) != 0;
    int rc = build_level_tables(*t, k, digits, o->tab, o->sampled);
    if (rc) {
        free_ops(o);
        return rc;
    }
    const int nl = t->n_lev;
    const int64_t R = max_rhs;
    const int64_t nleaf = t->lev[nl].nbox;
    // ---- plan the device bytes before touching the device
    Planner pl;
    pl.add(t->n * 16);                 // pts
    pl.add(t->n * 4 * 2);              // perm, pt_leaf
    pl.add((nleaf + 1) * 4 * 2);       // pt_start, near_start
    pl.add((int64_t)t->near_idx.size() * 4);
    pl.add(nleaf * 12);
    pl.add((t->n / 64 + nleaf + 1) * 8);  // P2P work items
    pl.add(t->n * R * 8);              // qs
    pl.add(t->n * R * 8 * 3);          // near (3 components for the field)
    pl.add(t->n * R * 8 * 3 * 2);      // two fields for the position gradient
    int64_t scratch = 0;
    if (nl >= 3) {
        for (int l = 3; l <= nl; ++l) {
            const LevelTables &T = o->tab[l];
            const HostLevel &H = t->lev[l];
            pl.add(T.K * 16);
            if (o->sampled)
                pl.add((int64_t)T.Tsamp.size() * 4 + (int64_t)T.xr.size() * 4 +
                       (int64_t)T.trig64.size() * 8);
            else
                pl.add((int64_t)T.ntypes * T.K * 8);
            pl.add((H.nbox + 1) * 4);
            pl.add((int64_t)H.far_src.size() * 6);
            pl.add(H.nbox * 5);
            pl.add((H.nbox + 1) * 4);
            pl.add(H.nbox * 4 + 343 * 2 + (H.nbox + 1) * 4 + 26 * H.nbox * 4);
            pl.add((int64_t)H.far_src.size() * 36 + (H.nbox + 1) * 4);  // M2L records (bound)
            if (!o->sampled) {
                pl.add((int64_t)H.far_src.size() * 32);                 // antipodal record slots
                pl.add(((int64_t)T.ntypes + 1) * (T.K / 2 + 64) * 8 + (T.K + 64) * 4);  // Tp
                pl.add((int64_t)H.far_src.size() * 32);                 // octant record slots
                pl.add(57 * (8 * T.K + 64) * 8 + (8 * T.K + 64) * 4);   // To, operm (bound)
            }
            pl.add(H.nbox * R * T.K * 8 * 2);
            if (l < nl) {
                const LevelTables &C = o->tab[l + 1];
                pl.add(8 * T.K * 8);
                pl.add((int64_t)T.shift_axis.size() * 4);
                pl.add(((int64_t)T.iF.size() + T.iA.size() + T.iG.size() + T.aF.size() +
                        T.aB.size() + T.aG.size()) * 4);
                // pair kernel (BF16x3 fragments: up to 4x the FP32 ones)
                pl.add(2 * (H.nbox + 1) * 8 + 2 * 4 * ((int64_t)T.iF.size() + T.iA.size() +
                                                      T.iG.size() + 64 * 64) *
                                                     ((flags & MLFMA_BF16X3_INTERP) ? 4 : 1));
                const int64_t e = t->lev[l + 1].nbox * R * std::max(C.nth, T.nth) * T.Mc;
                scratch = std::max(scratch, e);
            }
        }
        pl.add(scratch * 8 * 2);
    }
    o->planned_bytes = pl.bytes;
    const int64_t lim = g_mem_limit.load();
    if (lim > 0 && pl.bytes > lim) {
        rc = fail(MLFMA_ENOMEM, "precompute: needs %lld device bytes, limit is %lld",
                  (long long)pl.bytes, (long long)lim);
        free_ops(o);
        return rc;
    }
    // ---- device
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(o->device) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(MLFMA_EDEVICE, "precompute: cannot use HIP device %d", o->device);
        free_ops(o);
        return rc;
    }
    rc = [&]() -> int {
        int r;
        std::vector<float4> p = point_offsets(*t);
        if ((r = upload(o, &o->pts, p.data(), t->n))) return r;
        std::vector<int32_t> v32(t->perm.begin(), t->perm.end());
        if ((r = upload(o, &o->perm, v32.data(), t->n))) return r;
        if ((r = upload(o, &o->pt_leaf, t->pt_leaf.data(), t->n))) return r;
        v32.assign(t->pt_start.begin(), t->pt_start.end());
        if ((r = upload(o, &o->pt_start, v32.data(), (int64_t)v32.size()))) return r;
        v32.assign(t->near_start.begin(), t->near_start.end());
        if ((r = upload(o, &o->near_start, v32.data(), (int64_t)v32.size()))) return r;
        if ((r = upload(o, &o->near_idx, t->near_idx.data(), (int64_t)t->near_idx.size()))) return r;
        if ((r = upload(o, &o->leaf_coord, t->lev[nl].coord.data(), 3 * nleaf))) return r;
        // P2P work items, heavy ones (many target x source pairs: dense
        // leaves) first; those run with four waves per item
        std::vector<int2> items, light;
        for (int64_t b = 0; b < nleaf; ++b) {
            int64_t nsrc = 0;
            for (int64_t e = t->near_start[b]; e < t->near_start[b + 1]; ++e) {
                const int32_t nb = t->near_idx[e];
                nsrc += t->pt_start[nb + 1] - t->pt_start[nb];
            }
            const int64_t np = t->pt_start[b + 1] - t->pt_start[b];
            for (int64_t t0 = 0; t0 < np; t0 += 64) {
                const int64_t nt = std::min<int64_t>(64, np - t0);
                (nt * nsrc >= (int64_t)1 << 15 ? items : light).push_back(make_int2((int)b, (int)t0));
            }
        }
        o->n_p2p_heavy = (int64_t)items.size();
        items.insert(items.end(), light.begin(), light.end());
        o->n_p2p_items = (int64_t)items.size();
        if ((r = upload(o, &o->p2p_items, items.data(), o->n_p2p_items))) return r;
        if ((r = dalloc(o, &o->qs, t->n * R))) return r;
        if ((r = dalloc(o, &o->near, t->n * R * 3))) return r;
        if ((r = dalloc(o, &o->fq, t->n * R * 3))) return r;
        if ((r = dalloc(o, &o->fg, t->n * R * 3))) return r;
        o->lev.resize(nl + 1);
        for (int l = 1; l <= nl; ++l) o->lev[l].nbox = t->lev[l].nbox;
        if (nl < 3) return MLFMA_OK;
        // parents of the far-field levels: child ranges and neighbour lists
        for (int l = 2; l < nl; ++l) {
            DevLevel &D = o->lev[l];
            const HostLevel &H = t->lev[l];
            if ((r = upload(o, &D.child_start, H.child_start.data(), H.nbox + 1))) return r;
            std::vector<int32_t> ns, ni;
            neighbour_lists(*t, l, ns, ni);
            if ((r = upload(o, &D.nbr_start, ns.data(), (int64_t)ns.size()))) return r;
            if ((r = upload(o, &D.nbr_idx, ni.data(), (int64_t)ni.size()))) return r;
        }
        for (int l = 3; l <= nl; ++l) {
            DevLevel &D = o->lev[l];
            const LevelTables &T = o->tab[l];
            const HostLevel &H = t->lev[l];
            D.L = T.L;
            D.nth = T.nth;
            D.nph = T.nph;
            D.K = T.K;
            D.ntypes = T.ntypes;
            D.n_far = (int64_t)H.far_src.size();
            if ((r = upload(o, &D.khat_w, (const float4 *)T.khat_w.data(), T.K))) return r;
            if (o->sampled) {
                if ((r = upload(o, &D.Tsamp, (const float2 *)T.Tsamp.data(),
                                (int64_t)T.Tsamp.size() / 2)))
                    return r;
                if ((r = upload(o, &D.xr, (const float4 *)T.xr.data(), (int64_t)T.ntypes)))
                    return r;
                if ((r = upload(o, &D.trig64, T.trig64.data(), (int64_t)T.trig64.size())))
                    return r;
                D.Msamp = T.Msamp;
                D.m2l_variant = 5;
                o->operator_bytes += (int64_t)(T.Tsamp.size() + T.xr.size()) * 4 +
                                     (int64_t)T.trig64.size() * 8;
            } else {
                if ((r = upload(o, &D.T, (const float2 *)T.T.data(), (int64_t)T.ntypes * T.K)))
                    return r;
                o->operator_bytes += (int64_t)T.ntypes * T.K * 8;
            }
            if ((r = upload(o, &D.far_start, H.far_start.data(), H.nbox + 1))) return r;
            if ((r = upload(o, &D.far_src, H.far_src.data(), D.n_far))) return r;
            if ((r = upload(o, &D.far_type, T.far_type.data(), D.n_far))) return r;
            if ((r = upload(o, &D.parent, H.parent.data(), H.nbox))) return r;
            std::vector<uint8_t> oc(H.nbox);
            for (int64_t b = 0; b < H.nbox; ++b)
                oc[b] = (uint8_t)(((H.coord[3 * b] & 1) << 2) | ((H.coord[3 * b + 1] & 1) << 1) |
                                  (H.coord[3 * b + 2] & 1));
            if ((r = upload(o, &D.oct, oc.data(), H.nbox))) return r;
            if ((r = dalloc(o, &D.S, H.nbox * R * T.K))) return r;
            if ((r = dalloc(o, &D.Lloc, H.nbox * R * T.K))) return r;
            {
                // per-source records of the parents (level l-1) of this level
                const HostLevel &HP = t->lev[l - 1];
                std::vector<int32_t> ns, ni;
                neighbour_lists(*t, l - 1, ns, ni);
                std::vector<int32_t> rs(HP.nbox + 1, 0), rsrc, roff;
                const int32_t zero_row = T.ntypes * 64 * (int32_t)sizeof(float2);
                for (int64_t p = 0; p < HP.nbox; ++p) {
                    const int32_t o0 = HP.child_start[p], o1 = HP.child_start[p + 1];
                    for (int32_t e = ns[p]; e < ns[p + 1]; ++e) {
                        const int32_t q = ni[e];
                        for (int32_t sb = HP.child_start[q]; sb < HP.child_start[q + 1]; ++sb) {
                            uint16_t ty[8];
                            bool any = false;
                            for (int i = 0; i < 8; ++i) {
                                ty[i] = 0xffff;
                                if (o0 + i >= o1) continue;
                                const int32_t *co = &H.coord[3 * (o0 + i)], *cs = &H.coord[3 * sb];
                                const int dx = co[0] - cs[0], dy = co[1] - cs[1], dz = co[2] - cs[2];
                                if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) < 2)
                                    continue;
                                const int code = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
                                const int16_t tt = T.code_to_type[code];
                                if (tt >= 0) {
                                    ty[i] = (uint16_t)tt;
                                    any = true;
                                }
                            }
                            if (!any) continue;
                            rsrc.push_back(sb);
                            for (int i = 0; i < 8; ++i)
                                roff.push_back(ty[i] == 0xffff ? zero_row
                                                               : (int32_t)ty[i] * 64 * (int32_t)sizeof(float2));
                        }
                    }
                    // pad the parent's records to a multiple of 4 with records
                    // that add zero (the last source again, every slot on the
                    // zero row), so the kernel walks them in whole batches
                    while ((rsrc.size() - (size_t)rs[p]) % 4 != 0) {
                        rsrc.push_back(rsrc.back());
                        for (int i = 0; i < 8; ++i) roff.push_back(zero_row);
                    }
                    rs[p + 1] = (int32_t)rsrc.size();
                }
                // 8 zero records after the last list: the kernel's pipeline
                // fetches up to two batches of 4 past the end of a list
                for (int u = 0; u < 8; ++u) {
                    rsrc.push_back(0);
                    for (int i = 0; i < 8; ++i) roff.push_back(zero_row);
                }
                if ((r = upload(o, &D.rec_start, rs.data(), (int64_t)rs.size()))) return r;
                if ((r = upload(o, &D.rec_src, rsrc.data(), (int64_t)rsrc.size()))) return r;
                if ((r = upload(o, &D.rec_off, roff.data(), (int64_t)roff.size()))) return r;
                // the antipodal and octant forms copy from the full table
                if (!o->sampled) {
                    // antipodal slices: the opposite of sample (i, j) is
                    // (nth - 1 - i, j + nph / 2); T_{-d}(k) = T_d(-k)
                    const int64_t K = T.K;
                    auto anti = [&](int64_t q) -> int64_t {
                        const int64_t i = q / T.nph, j = q % T.nph;
                        return (T.nth - 1 - i) * T.nph + (j + T.nph / 2) % T.nph;
                    };
                    std::vector<int64_t> canon;
                    for (int64_t q = 0; q < K; ++q)
                        if (q < anti(q)) canon.push_back(q);
                    const int64_t npair = (int64_t)canon.size();
                    const int64_t nsl = (npair + 31) / 32;
                    D.Kp = nsl * 64;
                    std::vector<int32_t> ap((size_t)D.Kp, -1);
                    for (int64_t sl = 0; sl < nsl; ++sl)
                        for (int ln = 0; ln < 32; ++ln) {
                            const int64_t pr = sl * 32 + ln;
                            if (pr >= npair) break;
                            ap[(size_t)(sl * 64 + ln)] = (int32_t)canon[(size_t)pr];
                            ap[(size_t)(sl * 64 + 63 - ln)] = (int32_t)anti(canon[(size_t)pr]);
                        }
                    // offset pairs: code(-d) = 342 - code(d); the smaller code
                    // of a used pair names it
                    std::vector<int> tp_of(343, -1), type_code(T.ntypes, -1);
                    int ntp = 0;
                    for (int c = 0; c < 343; ++c) {
                        if (T.code_to_type[c] < 0) continue;
                        type_code[T.code_to_type[c]] = c;
                        const int c0 = std::min(c, 342 - c);
                        if (tp_of[c0] < 0) tp_of[c0] = ntp++;
                    }
                    D.ntp = ntp;
                    std::vector<float2> tpv((size_t)ntp * D.Kp, make_float2(0.f, 0.f));
                    const float2 *Th = (const float2 *)T.T.data();
                    for (int c0 = 0; c0 < 343; ++c0) {
                        if (tp_of[c0] < 0) continue;
                        // the row of offset c0, or the mirrored row of -c0
                        const bool direct = T.code_to_type[c0] >= 0;
                        const int t = direct ? T.code_to_type[c0] : T.code_to_type[342 - c0];
                        for (int64_t e = 0; e < D.Kp; ++e) {
                            const int32_t q = ap[(size_t)e];
                            if (q < 0) continue;
                            tpv[(size_t)tp_of[c0] * D.Kp + e] = Th[(size_t)t * K + (direct ? q : anti(q))];
                        }
                    }
                    std::vector<int32_t> ranti(roff.size());
                    for (size_t e = 0; e < roff.size(); ++e) {
                        if (roff[e] == zero_row) {
                            ranti[e] = ntp * 512;
                            continue;
                        }
                        const int c = type_code[roff[e] / (64 * (int32_t)sizeof(float2))];
                        const int c0 = std::min(c, 342 - c);
                        ranti[e] = tp_of[c0] * 512 | (c != c0 ? 504 : 0);
                    }
                    if ((r = upload(o, &D.Tp, tpv.data(), (int64_t)tpv.size()))) return r;
                    if ((r = upload(o, &D.aperm, ap.data(), D.Kp))) return r;
                    if ((r = upload(o, &D.rec_off_anti, ranti.data(), (int64_t)ranti.size()))) return r;

                    // octant slices: reflection g (bit 2: x, phi -> pi - phi;
                    // bit 1: y, phi -> -phi; bit 0: z, theta -> pi - theta) of
                    // sample q; the reflected offset R_g d has T_{R_g d}(q) =
                    // T_d(refl(g, q))
                    auto refl = [&](int g, int64_t q) -> int64_t {
                        int64_t i = q / T.nph, j = q % T.nph;
                        if (g & 1) i = T.nth - 1 - i;
                        if (g & 2) j = (T.nph - j) % T.nph;
                        if (g & 4) j = (T.nph / 2 - j + T.nph) % T.nph;
                        return i * T.nph + j;
                    };
                    std::vector<char> seen((size_t)K, 0);
                    std::vector<int64_t> orbit0;
                    for (int64_t q = 0; q < K; ++q) {
                        if (seen[(size_t)q]) continue;
                        orbit0.push_back(q);
                        for (int g = 0; g < 8; ++g) seen[(size_t)refl(g, q)] = 1;
                    }
                    const int64_t nso = ((int64_t)orbit0.size() + 7) / 8;
                    D.Ko = nso * 64;
                    std::vector<int32_t> opm((size_t)D.Ko, -1);
                    for (size_t ob = 0; ob < orbit0.size(); ++ob)
                        for (int g = 0; g < 8; ++g) {
                            const int64_t q = refl(g, orbit0[ob]);
                            bool first = true;
                            for (int h = 0; h < g; ++h)
                                if (refl(h, orbit0[ob]) == q) first = false;
                            opm[ob * 8 + g] = first ? (int32_t)q : (int32_t)(-q - 2);
                        }
                    // rows: the offsets (|dx|, |dy|, |dz|) of the used offsets
                    std::vector<int> row_of(64, -1), src_code(64, -1);
                    int nto = 0;
                    for (int c = 0; c < 343; ++c) {
                        if (T.code_to_type[c] < 0) continue;
                        const int dx = c / 49 - 3, dy = (c / 7) % 7 - 3, dz = c % 7 - 3;
                        const int a = std::abs(dx) * 16 + std::abs(dy) * 4 + std::abs(dz);
                        if (row_of[a] < 0) {
                            row_of[a] = nto++;
                            src_code[a] = c;
                        }
                    }
                    D.nto = nto;
                    std::vector<float2> tov((size_t)nto * D.Ko, make_float2(0.f, 0.f));
                    for (int a = 0; a < 64; ++a) {
                        if (row_of[a] < 0) continue;
                        const int c = src_code[a];
                        const int dx = c / 49 - 3, dy = (c / 7) % 7 - 3, dz = c % 7 - 3;
                        const int g = (dx < 0 ? 4 : 0) | (dy < 0 ? 2 : 0) | (dz < 0 ? 1 : 0);
                        const int t = T.code_to_type[c];
                        // T_{|d|}(q) = T_{R_g |d|}(refl(g, q)), R_g |d| = d
                        for (int64_t e = 0; e < D.Ko; ++e) {
                            const int32_t cd = opm[(size_t)e];
                            if (cd == -1) continue;
                            const int64_t q = cd >= 0 ? cd : -(int64_t)cd - 2;
                            tov[(size_t)row_of[a] * D.Ko + e] = Th[(size_t)t * K + refl(g, q)];
                        }
                    }
                    std::vector<int32_t> roct(roff.size());
                    for (size_t e = 0; e < roff.size(); ++e) {
                        if (roff[e] == zero_row) {
                            roct[e] = nto * 512;
                            continue;
                        }
                        const int c = type_code[roff[e] / (64 * (int32_t)sizeof(float2))];
                        const int dx = c / 49 - 3, dy = (c / 7) % 7 - 3, dz = c % 7 - 3;
                        const int a = std::abs(dx) * 16 + std::abs(dy) * 4 + std::abs(dz);
                        const int g = (dx < 0 ? 4 : 0) | (dy < 0 ? 2 : 0) | (dz < 0 ? 1 : 0);
                        roct[e] = row_of[a] * 512 | (g * 8);
                    }
                    if ((r = upload(o, &D.To, tov.data(), (int64_t)tov.size()))) return r;
                    if ((r = upload(o, &D.operm, opm.data(), D.Ko))) return r;
                    if ((r = upload(o, &D.rec_off_oct, roct.data(), (int64_t)roct.size()))) return r;
                    o->operator_bytes += ((int64_t)D.ntp * D.Kp + (int64_t)D.nto * D.Ko) * 8;
                }
            }
            {
                std::vector<int32_t> bs(H.nbox);
                for (int64_t b = 0; b < H.nbox; ++b)
                    bs[b] = 49 * H.coord[3 * b] + 7 * H.coord[3 * b + 1] + H.coord[3 * b + 2];
                if ((r = upload(o, &D.base, bs.data(), H.nbox))) return r;
                if ((r = upload(o, &D.typemap, T.code_to_type.data(), 343))) return r;
            }
            if (l < nl) {
                D.Lc = T.Lc;
                D.Mc = T.Mc;
                if ((r = upload(o, &D.shift, (const float2 *)T.shift.data(), 8 * T.K))) return r;
                if ((r = upload(o, &D.shift_axis, (const float2 *)T.shift_axis.data(),
                                (int64_t)T.shift_axis.size() / 2)))
                    return r;
                if ((r = upload(o, &D.iF, T.iF.data(), (int64_t)T.iF.size()))) return r;
                if ((r = upload(o, &D.iA, T.iA.data(), (int64_t)T.iA.size()))) return r;
                if ((r = upload(o, &D.iG, T.iG.data(), (int64_t)T.iG.size()))) return r;
                if ((r = upload(o, &D.aF, T.aF.data(), (int64_t)T.aF.size()))) return r;
                if ((r = upload(o, &D.aB, T.aB.data(), (int64_t)T.aB.size()))) return r;
                if ((r = upload(o, &D.aG, T.aG.data(), (int64_t)T.aG.size()))) return r;
            }
        }
        o->scratch_elems = scratch;
        if ((r = dalloc(o, &o->X1, scratch))) return r;
        if ((r = dalloc(o, &o->X2, scratch))) return r;
        // spectra start zeroed (the autotuner runs the kernels on them)
        for (int l = 3; l <= nl; ++l) {
            DevLevel &D = o->lev[l];
            if (hipMemset(D.S, 0, (size_t)(D.nbox * R * D.K) * sizeof(float2)) != hipSuccess ||
                hipMemset(D.Lloc, 0, (size_t)(D.nbox * R * D.K) * sizeof(float2)) != hipSuccess)
                return fail(MLFMA_EDEVICE, "hipMemset failed");
        }
        // one-pass interpolation where its LDS plan fits; FP32 path only
        for (int l = 3; l < nl; ++l) {
            DevLevel &P = o->lev[l], &C = o->lev[l + 1];
            P.onepass_ok = dev::pair_onepass_fits(C.L, P.L);
            const bool use = P.onepass_ok && !(flags & MLFMA_BF16X3_INTERP);
            P.interp_variant = use ? 1 : 0;
            P.anterp_variant = use ? 1 : 0;
        }
        // fused pair kernel (FP32 or BF16x3): parent groups and fragment tables
        for (int l = 3; l < nl; ++l) {
            DevLevel &P = o->lev[l], &C = o->lev[l + 1];
            const LevelTables &T = o->tab[l];
            const HostLevel &H = t->lev[l];
            for (int dn = 0; dn < 2; ++dn) {
                if (!dev::pair_kernel_fits(C.L, P.L, dn == 1)) continue;
                dev::PairTables pt;
                if (dev::pair_tables(C.L, P.L, dn == 1, dn ? T.aF.data() : T.iF.data(),
                                     dn ? T.aB.data() : T.iA.data(),
                                     dn ? T.aG.data() : T.iG.data(), &pt,
                                     (flags & MLFMA_BF16X3_INTERP) != 0))
                    return fail(MLFMA_EINVAL, "precompute: pair tables of level %d", l);
                // runs of whole parents with at most max_children (8)
                // children, each described by two int4 (see pair_map)
                const HostLevel &HC = t->lev[l + 1];
                std::vector<int4> tiles;
                for (int64_t p = 0; p < H.nbox;) {
                    int64_t q = p;
                    while (q < H.nbox && q - p < pt.max_parents &&
                           H.child_start[q + 1] - H.child_start[p] <= pt.max_children)
                        ++q;
                    const int cb = H.child_start[p], nb = H.child_start[q] - cb;
                    int octs = 0, ppf = 0, spar = 0;
                    for (int i = 0; i < nb; ++i) {
                        const int32_t *cc = &HC.coord[3 * (cb + i)];
                        const int oc = ((cc[0] & 1) << 2) | ((cc[1] & 1) << 1) | (cc[2] & 1);
                        octs |= oc << (3 * i);
                    }
                    for (int64_t j = 1; j < q - p; ++j)
                        ppf |= (H.child_start[p + j] - cb) << (4 * (j - 1));
                    for (int64_t j = 0; j < q - p; ++j)
                        for (int i = H.child_start[p + j] - cb; i < H.child_start[p + j + 1] - cb; ++i)
                            spar |= (int)j << (3 * i);
                    tiles.push_back(make_int4((int)p, cb, nb, (int)(q - p)));
                    tiles.push_back(make_int4(octs, ppf, spar, 0));
                    p = q;
                }
                P.nptile[dn] = (int64_t)tiles.size() / 2;
                if ((r = upload(o, &P.ptile[dn], tiles.data(), (int64_t)tiles.size()))) return r;
                if ((r = upload(o, &P.pfr[dn][0], pt.fr1.data(), (int64_t)pt.fr1.size()))) return r;
                if ((r = upload(o, &P.pfr[dn][1], pt.fr2.data(), (int64_t)pt.fr2.size()))) return r;
                if ((r = upload(o, &P.pfr[dn][2], pt.fr3.data(), (int64_t)pt.fr3.size()))) return r;
                P.pair_ok[dn] = true;
            }
        }
        if (!(flags & MLFMA_NO_AUTOTUNE)) {
            if ((r = autotune(o))) return r;
        }
        // streams and events of the concurrent schedule (default priority)
        if (!(flags & MLFMA_ONE_STREAM) && nl >= 3) {
            for (hipStream_t &st : o->side)
                if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
                    return fail(MLFMA_EDEVICE, "precompute: stream creation failed");
            // The fork and join events order kernels of this device only,
            // so they are recorded without the system-scope fence (the
            // producing kernel's own end-of-kernel release makes its
            // results visible to the other streams' kernels; with the
            // fence's cache write-back at each of the ~6 records a matvec
            // of the 262k sphere took 0.589 ms, without it 0.583 ms)
            constexpr unsigned kEvFlags = hipEventDisableTiming | hipEventDisableSystemFence;
            o->ev_S.assign(nl + 1, nullptr);
            for (hipEvent_t *e : {&o->ev_fork, &o->ev_near, &o->ev_m2l, &o->ev_leaf})
                if (hipEventCreateWithFlags(e, kEvFlags) != hipSuccess)
                    return fail(MLFMA_EDEVICE, "precompute: event creation failed");
            for (int l = 3; l <= nl; ++l)
                if (hipEventCreateWithFlags(&o->ev_S[l], kEvFlags) != hipSuccess)
                    return fail(MLFMA_EDEVICE, "precompute: event creation failed");
            if (!(flags & MLFMA_NO_AUTOTUNE)) {
                if ((r = tune_concurrent(o))) return r;
            }
        }
        return MLFMA_OK;
    }();
    (void)hipSetDevice(cur);
    if (rc) {
        free_ops(o);
        return rc;
    }
    o->pos_version = t->pos_version;
    *out = o;
    return MLFMA_OK;
}

int mlfma_matvec(mlfma_ops_t ops, const void *q, void *phi, int64_t nrhs, int dtype, void *stream)
{
    return do_matvec(ops, q, phi, nrhs, dtype, MLFMA_NEAR | MLFMA_FAR, 0, (hipStream_t)stream);
}

int mlfma_matvec_adjoint(mlfma_ops_t ops, const void *v, void *psi, int64_t nrhs, int dtype,
                         void *stream)
{
    return do_matvec(ops, v, psi, nrhs, dtype, MLFMA_NEAR | MLFMA_FAR | MLFMA_CONJ, 0,
                     (hipStream_t)stream);
}

int mlfma_matvec_ex(mlfma_ops_t ops, const void *q, void *phi, int64_t nrhs, int dtype,
                    uint32_t parts, void *stream)
{
    return do_matvec(ops, q, phi, nrhs, dtype, parts, 0, (hipStream_t)stream);
}

// ----------------------------------------------------------- GMRES solve --
namespace {

static void free_alloc(mlfma_ops_s *o, void *p)
{
    if (!p) return;
    auto it = std::find(o->allocs.begin(), o->allocs.end(), p);
    if (it != o->allocs.end()) o->allocs.erase(it);
    (void)hipFree(p);
}

static int gm_workspace(mlfma_ops_s *o, int m)
{
    if (m <= o->gm_cap) return MLFMA_OK;
    free_alloc(o, o->gm_V);
    free_alloc(o, o->gm_w);
    free_alloc(o, o->gm_part);
    free_alloc(o, o->gm_c);
    o->gm_V = o->gm_w = nullptr;
    o->gm_part = o->gm_c = nullptr;
    o->gm_cap = 0;
    const int64_t n = o->n, nb = dev::gm_dot_blocks(n);
    const int64_t bytes = ((int64_t)(m + 2) * n) * (int64_t)sizeof(float2) +
                          (int64_t)(m + 1) * nb * (int64_t)sizeof(double2) +
                          (int64_t)(m + 1) * (int64_t)sizeof(double2);
    const int64_t lim = g_mem_limit.load();
    if (lim > 0 && o->planned_bytes + bytes > lim)
        return fail(MLFMA_ENOMEM, "solve_gmres: workspace of %lld bytes exceeds the limit of %lld",
                    (long long)bytes, (long long)lim);
    int r;
    if ((r = dalloc(o, &o->gm_V, (int64_t)(m + 1) * n))) return r;
    if ((r = dalloc(o, &o->gm_w, n))) return r;
    if ((r = dalloc(o, &o->gm_part, (int64_t)(m + 1) * nb))) return r;
    if ((r = dalloc(o, &o->gm_c, (int64_t)(m + 1)))) return r;
    o->gm_cap = m;
    return MLFMA_OK;
}

// Device scratch of the allocation-free solve: one array per GPU, placed by
// the code-object loader (no hipMalloc).  Host code never passes the
// array's name to a kernel or a copy: it takes the device address that
// hipGetSymbolAddress returns, once per device, and uses only that.
static __device__ __align__(256) unsigned char scratch[MLFMA_GMRES_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current.
static int scratch_address(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(MLFMA_EDEVICE, "solve_gmres_noalloc: device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(MLFMA_EDEVICE, "solve_gmres_noalloc: hipGetSymbolAddress(scratch): %s",
                        hipGetErrorString(e));
        }
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[device]);
    return MLFMA_OK;
}

struct GmBuffers {
    float2 *V = nullptr, *w = nullptr;
    double2 *part = nullptr, *c = nullptr;
};

static int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// The GMRES buffers of restart m carved from the device scratch:
// V [(m + 1) x n], w [n] complex64, block partials [(m + 1) x nb] and
// coefficients [m + 1] complex FP64, each at a 256-byte boundary.
static int gm_static(mlfma_ops_s *o, int m, GmBuffers *out)
{
    const int64_t n = o->n, nb = dev::gm_dot_blocks(n);
    const int64_t bV = align256((int64_t)(m + 1) * n * (int64_t)sizeof(float2));
    const int64_t bw = align256(n * (int64_t)sizeof(float2));
    const int64_t bp = align256((int64_t)(m + 1) * nb * (int64_t)sizeof(double2));
    const int64_t bc = align256((int64_t)(m + 1) * (int64_t)sizeof(double2));
    const int64_t need = bV + bw + bp + bc;
    if (need > (int64_t)MLFMA_GMRES_SCRATCH_BYTES)
        return fail(MLFMA_ENOMEM,
                    "solve_gmres_noalloc: n = %lld with restart %d needs %lld bytes of "
                    "scratch, more than the fixed %lld",
                    (long long)n, m, (long long)need, (long long)MLFMA_GMRES_SCRATCH_BYTES);
    unsigned char *base = nullptr;
    if (int r = scratch_address(o->device, &base)) return r;
    out->V = reinterpret_cast<float2 *>(base);
    out->w = reinterpret_cast<float2 *>(base + bV);
    out->part = reinterpret_cast<double2 *>(base + bV + bw);
    out->c = reinterpret_cast<double2 *>(base + bV + bw + bp);
    return MLFMA_OK;
}

static int gmres_run(mlfma_ops_t o, const void *b, void *x, double shift_re, double shift_im,
              int restart, int max_iters, double tol, int *iters, double *rel_residual,
              void *stream, bool noalloc)
{
    typedef std::complex<double> cd;
    if (iters) *iters = 0;
    if (rel_residual) *rel_residual = 0.0;
    if (restart < 1 || restart > 500)
        return fail(MLFMA_EINVAL, "solve_gmres: restart %d outside 1..500", restart);
    if (max_iters < 0) return fail(MLFMA_EINVAL, "solve_gmres: max_iters < 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MLFMA_EINVAL, "solve_gmres: tol must be > 0");
    if (!std::isfinite(shift_re) || !std::isfinite(shift_im))
        return fail(MLFMA_EINVAL, "solve_gmres: shift is not finite");
    if (!o) return fail(MLFMA_EINVAL, "solve_gmres: ops handle is NULL");
    if (o->n == 0) return MLFMA_OK;
    if (!b || !x) return fail(MLFMA_EINVAL, "solve_gmres: null buffer");
    if (b == x) return fail(MLFMA_EINVAL, "solve_gmres: b and x must not alias");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(MLFMA_EDEVICE, "hipGetDevice failed");
    if (cur != o->device && hipSetDevice(o->device) != hipSuccess)
        return fail(MLFMA_EDEVICE, "hipSetDevice(%d) failed", o->device);
    const int m = restart;
    GmBuffers wb;
    int rc = MLFMA_OK;
    if (noalloc) {
        rc = gm_static(o, m, &wb);
    } else {
        rc = gm_workspace(o, m);
        wb.V = o->gm_V;
        wb.w = o->gm_w;
        wb.part = o->gm_part;
        wb.c = o->gm_c;
    }
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = o->n;
    const int nb = dev::gm_dot_blocks(n);
    const float2 *bv = (const float2 *)b;
    float2 *xv = (float2 *)x, *V = wb.V, *w = wb.w;
    double2 *gpart = wb.part, *gcoef = wb.c;
    auto row = [&](int i) { return V + (int64_t)i * n; };
    std::vector<double2> part((size_t)(m + 1) * nb), coef(m + 1);
    // out[i] = <V_i, u> for i < cnt (FP64 sums of the block partials)
    auto dots = [&](const float2 *Vb, int cnt, const float2 *u, cd *out) -> int {
        CK(dev::gm_dots(Vb, n, cnt, u, n, nb, gpart, s));
        CK(hipMemcpyAsync(part.data(), gpart, (size_t)cnt * nb * sizeof(double2),
                          hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        for (int i = 0; i < cnt; ++i) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < nb; ++k) {
                re += part[(size_t)i * nb + k].x;
                im += part[(size_t)i * nb + k].y;
            }
            out[i] = cd(re, im);
        }
        return MLFMA_OK;
    };
    // out[i] = <V_i, u> for i < cnt and *uu = <u, u>, one host round trip
    auto dots_norm = [&](int cnt, const float2 *u, cd *out, double *uu) -> int {
        CK(dev::gm_dots(V, n, cnt, u, n, nb, gpart, s));
        CK(dev::gm_dots(u, n, 1, u, n, nb, gpart + (size_t)cnt * nb, s));
        CK(hipMemcpyAsync(part.data(), gpart, (size_t)(cnt + 1) * nb * sizeof(double2),
                          hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        for (int i = 0; i <= cnt; ++i) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < nb; ++k) {
                re += part[(size_t)i * nb + k].x;
                im += part[(size_t)i * nb + k].y;
            }
            if (i < cnt) out[i] = cd(re, im);
            else *uu = re;
        }
        return MLFMA_OK;
    };
    auto norm = [&](const float2 *u, double *out) -> int {
        cd d;
        if (int r = dots(u, 1, u, &d)) return r;
        *out = std::sqrt(std::max(0.0, d.real()));
        return MLFMA_OK;
    };
    // u <- u + sign * sum_{i < cnt} V_i c_i
    auto combine = [&](float2 *u, int cnt, const cd *c, double sign) -> int {
        for (int i = 0; i < cnt; ++i) coef[i] = make_double2(c[i].real(), c[i].imag());
        CK(hipMemcpyAsync(gcoef, coef.data(), (size_t)cnt * sizeof(double2),
                          hipMemcpyHostToDevice, s));
        CK(dev::gm_combine(u, V, n, cnt, gcoef, sign, n, s));
        return MLFMA_OK;
    };
    // y <- (shift I + A) v
    auto op = [&](const float2 *v, float2 *y) -> int {
        // eager: the solver's operands cycle through the basis rows, more
        // buffer pairs than the graph cache holds
        if (int r = do_matvec(o, v, y, 1, MLFMA_C64, MLFMA_NEAR | MLFMA_FAR, 0, s, -1, -1, -1,
                              false))
            return r;
        CK(dev::gm_axpby(y, make_double2(shift_re, shift_im), v, make_double2(1.0, 0.0), n, s));
        return MLFMA_OK;
    };
    double bnorm = 0.0;
    if ((rc = norm(bv, &bnorm))) return rc;
    if (bnorm == 0.0) {
        CK(dev::gm_axpby(xv, make_double2(0.0, 0.0), xv, make_double2(0.0, 0.0), n, s));
        CK(hipStreamSynchronize(s));
        return MLFMA_OK;
    }
    std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), h(m + 1), y(m);
    auto Hat = [&](int i, int j) -> cd & { return H[(size_t)i * m + j]; };
    int total = 0;
    double relres = 0.0;
    for (;;) {
        // true residual r = b - (shift I + A) x in V_0
        if ((rc = op(xv, w))) return rc;
        CK(dev::gm_axpby(row(0), make_double2(1.0, 0.0), bv, make_double2(0.0, 0.0), n, s));
        CK(dev::gm_axpby(row(0), make_double2(-1.0, 0.0), w, make_double2(1.0, 0.0), n, s));
        double beta = 0.0;
        if ((rc = norm(row(0), &beta))) return rc;
        relres = beta / bnorm;
        if (relres <= tol || total >= max_iters || beta == 0.0) break;
        CK(dev::gm_axpby(row(0), make_double2(1.0 / beta, 0.0), row(0), make_double2(0.0, 0.0), n, s));
        std::fill(g.begin(), g.end(), cd(0.0));
        std::fill(H.begin(), H.end(), cd(0.0));
        g[0] = beta;
        int j = 0;
        for (; j < m && total < max_iters;) {
            if ((rc = op(row(j), w))) return rc;
            ++total;
            // classical Gram-Schmidt, repeated once when the projection
            // removed most of w (norm ratio below 1/sqrt(2): "twice is
            // enough", Kahan and Parlett), so the basis stays orthonormal
            // (the norm after a pass is ||w||^2 - sum |h_i|^2 for the
            // orthonormal basis; the repeated pass measures it directly)
            double ww = 0.0, hn = 0.0;
            if ((rc = dots_norm(j + 1, w, h.data(), &ww))) return rc;
            if ((rc = combine(w, j + 1, h.data(), -1.0))) return rc;
            double hh = 0.0;
            for (int i = 0; i <= j; ++i) {
                Hat(i, j) += h[i];
                hh += std::norm(h[i]);
            }
            if (ww - hh > 0.5 * ww) {
                hn = std::sqrt(ww - hh);
            } else {
                if ((rc = dots(V, j + 1, w, h.data()))) return rc;
                if ((rc = combine(w, j + 1, h.data(), -1.0))) return rc;
                for (int i = 0; i <= j; ++i) Hat(i, j) += h[i];
                if ((rc = norm(w, &hn))) return rc;
            }
            Hat(j + 1, j) = hn;
            if (hn > 0.0)
                CK(dev::gm_axpby(row(j + 1), make_double2(1.0 / hn, 0.0), w, make_double2(0.0, 0.0),
                                 n, s));
            // previous rotations on column j, then the one that zeroes H[j+1][j]
            for (int i = 0; i < j; ++i) {
                const cd a = Hat(i, j), c = Hat(i + 1, j);
                Hat(i, j) = cs[i] * a + sn[i] * c;
                Hat(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * c;
            }
            const cd a = Hat(j, j), c = Hat(j + 1, j);
            const double t = std::sqrt(std::norm(a) + std::norm(c));
            if (std::abs(a) == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
            } else {
                cs[j] = std::abs(a) / t;
                sn[j] = (a / std::abs(a)) * std::conj(c) / t;
            }
            Hat(j, j) = cs[j] * a + sn[j] * c;
            Hat(j + 1, j) = 0.0;
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            ++j;
            if (std::abs(g[j]) / bnorm <= tol || hn == 0.0) break;
        }
        // x += V y, H y = g (upper triangular, j columns)
        for (int i = j - 1; i >= 0; --i) {
            cd acc = g[i];
            for (int k = i + 1; k < j; ++k) acc -= Hat(i, k) * y[k];
            y[i] = Hat(i, i) != 0.0 ? acc / Hat(i, i) : cd(0.0);
        }
        if (j > 0)
            if ((rc = combine(xv, j, y.data(), 1.0))) return rc;
    }
    CK(hipStreamSynchronize(s));
    if (iters) *iters = total;
    if (rel_residual) *rel_residual = relres;
    return MLFMA_OK;
}

}  // namespace

int mlfma_solve_gmres(mlfma_ops_t o, const void *b, void *x, double shift_re, double shift_im,
                      int restart, int max_iters, double tol, int *iters, double *rel_residual,
                      void *stream)
{
    return gmres_run(o, b, x, shift_re, shift_im, restart, max_iters, tol, iters, rel_residual,
                     stream, false);
}

int mlfma_solve_gmres_noalloc(mlfma_ops_t o, const void *b, void *x, double shift_re,
                              double shift_im, int restart, int max_iters, double tol,
                              int *iters, double *rel_residual, void *stream)
{
    return gmres_run(o, b, x, shift_re, shift_im, restart, max_iters, tol, iters, rel_residual,
                     stream, true);
}

int mlfma_field(mlfma_ops_t ops, const void *q, void *grad, int64_t nrhs, int dtype,
                uint32_t parts, void *stream)
{
    return do_matvec(ops, q, grad, nrhs, dtype, parts, 1, (hipStream_t)stream);
}

int mlfma_position_gradient(mlfma_ops_t o, const void *q, const void *g, void *out, int64_t nrhs,
                            int dtype, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (!o) return fail(MLFMA_EINVAL, "position_gradient: ops is NULL");
    if (o->n > 0 && (!q || !g || !out)) return fail(MLFMA_EINVAL, "position_gradient: null buffer");
    // F_q and F_conj(g) into the workspace, both complex64 in caller order
    int rc = do_matvec(o, q, o->fq, nrhs, dtype, 0, 1, s, 0, 0, MLFMA_C64);
    if (rc) return rc;
    rc = do_matvec(o, g, o->fg, nrhs, dtype, 0, 1, s, 1, 0, MLFMA_C64);
    if (rc) return rc;
    if (o->n == 0) return MLFMA_OK;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(MLFMA_EDEVICE, "hipGetDevice failed");
    if (cur != o->device) (void)hipSetDevice(o->device);
    hipError_t e = dev::position_grad_combine(q, g, dtype, o->fq, o->fg, o->n, (int)nrhs, out, s);
    if (cur != o->device) (void)hipSetDevice(cur);
    return check_hip(e, "position_grad_combine");
}

void mlfma_destroy_ops(mlfma_ops_t ops) { free_ops(ops); }

void mlfma_destroy_tree(mlfma_tree_t t) { release_tree(reinterpret_cast<Tree *>(t)); }

int mlfma_tree_info_get(mlfma_tree_t th, mlfma_tree_info *out)
{
    Tree *t = reinterpret_cast<Tree *>(th);
    if (!t || !out) return fail(MLFMA_EINVAL, "tree_info: null argument");
    std::memset(out, 0, sizeof *out);
    out->n_points = t->n;
    out->n_levels = t->n_lev;
    out->device = t->device;
    out->leaf_size = t->leaf;
    out->root_size = t->D0;
    for (int a = 0; a < 3; ++a) out->origin[a] = t->origin[a];
    out->n_leaf_boxes = t->lev[t->n_lev].nbox;
    out->n_near_pairs = (int64_t)t->near_idx.size();
    out->n_p2p_pairs = t->n_p2p_pairs;
    return MLFMA_OK;
}

int mlfma_tree_permutation(mlfma_tree_t th, int64_t *perm)
{
    Tree *t = reinterpret_cast<Tree *>(th);
    if (!t || (!perm && t->n > 0)) return fail(MLFMA_EINVAL, "tree_permutation: null argument");
    std::memcpy(perm, t->perm.data(), t->perm.size() * sizeof(int64_t));
    return MLFMA_OK;
}

int mlfma_tree_level(mlfma_tree_t th, int level, int64_t *nbox, int32_t *coords,
                     int32_t *parent)
{
    Tree *t = reinterpret_cast<Tree *>(th);
    if (!t || !nbox) return fail(MLFMA_EINVAL, "tree_level: null argument");
    if (level < 1 || level > t->n_lev) return fail(MLFMA_EINVAL, "tree_level: bad level %d", level);
    const HostLevel &L = t->lev[level];
    *nbox = L.nbox;
    if (coords) std::memcpy(coords, L.coord.data(), L.coord.size() * sizeof(int32_t));
    if (parent) std::memcpy(parent, L.parent.data(), L.parent.size() * sizeof(int32_t));
    return MLFMA_OK;
}

int mlfma_tree_far_list(mlfma_tree_t th, int level, int64_t *count, int32_t *obs, int32_t *src,
                        int32_t *code)
{
    Tree *t = reinterpret_cast<Tree *>(th);
    if (!t || !count) return fail(MLFMA_EINVAL, "tree_far_list: null argument");
    if (level < 3 || level > t->n_lev)
        return fail(MLFMA_EINVAL, "tree_far_list: bad level %d", level);
    const HostLevel &L = t->lev[level];
    *count = (int64_t)L.far_src.size();
    for (int64_t b = 0; b < L.nbox; ++b)
        for (int32_t e = L.far_start[b]; e < L.far_start[b + 1]; ++e) {
            if (obs) obs[e] = (int32_t)b;
            if (src) src[e] = L.far_src[e];
            if (code) code[e] = L.far_code[e];
        }
    return MLFMA_OK;
}

int mlfma_tree_near_list(mlfma_tree_t th, int64_t *start, int32_t *idx)
{
    Tree *t = reinterpret_cast<Tree *>(th);
    if (!t) return fail(MLFMA_EINVAL, "tree_near_list: tree is NULL");
    if (start) std::memcpy(start, t->near_start.data(), t->near_start.size() * sizeof(int64_t));
    if (idx) std::memcpy(idx, t->near_idx.data(), t->near_idx.size() * sizeof(int32_t));
    return MLFMA_OK;
}

int mlfma_ops_info(mlfma_ops_t o, mlfma_level_info *out, int max_entries)
{
    if (!o || !out) return fail(MLFMA_EINVAL, "ops_info: null argument");
    const Tree *t = o->tree;
    for (int l = 1; l <= t->n_lev && l <= max_entries; ++l) {
        mlfma_level_info &I = out[l - 1];
        std::memset(&I, 0, sizeof I);
        I.level = l;
        I.nbox = t->lev[l].nbox;
        if (l >= 3) {
            const LevelTables &T = o->tab[l];
            I.L = T.L;
            I.ntheta = T.nth;
            I.nphi = T.nph;
            I.K = T.K;
            I.n_far = (int64_t)t->lev[l].far_src.size();
            I.n_types = T.ntypes;
        }
    }
    return MLFMA_OK;
}

int mlfma_copy_spectra(mlfma_ops_t o, int level, int which, int64_t nrhs, void *dst, void *stream)
{
    if (!o || !dst) return fail(MLFMA_EINVAL, "copy_spectra: null argument");
    if (level < 3 || level > o->n_lev) return fail(MLFMA_EINVAL, "copy_spectra: bad level");
    if (nrhs < 1 || nrhs > o->max_rhs) return fail(MLFMA_EINVAL, "copy_spectra: bad nrhs");
    const DevLevel &D = o->lev[level];
    const float2 *src = which == 0 ? D.S : D.Lloc;
    hipError_t e = hipMemcpyAsync(dst, src, (size_t)(D.nbox * nrhs * D.K) * sizeof(float2),
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return check_hip(e, "copy_spectra");
}

int mlfma_ops_variants(mlfma_ops_t o, int kernel, int32_t *out, int max_entries)
{
    if (!o || !out) return fail(MLFMA_EINVAL, "ops_variants: null argument");
    if (kernel == MLFMA_K_M2L) {
        for (int l = 1; l <= o->n_lev && l <= max_entries; ++l)
            out[l - 1] = l >= 3 ? o->lev[l].m2l_variant : -1;
        return MLFMA_OK;
    }
    if (kernel == MLFMA_K_INTERP || kernel == MLFMA_K_ANTERP) {
        for (int l = 1; l <= o->n_lev && l <= max_entries; ++l)
            out[l - 1] = (l >= 3 && l < o->n_lev)
                             ? (kernel == MLFMA_K_INTERP ? o->lev[l].interp_variant
                                                         : o->lev[l].anterp_variant)
                             : -1;
        return MLFMA_OK;
    }
    if (kernel == MLFMA_K_P2P) {
        if (max_entries >= 1) out[0] = o->side[0] ? o->near_fork : -1;
        if (max_entries >= 2) out[1] = o->side[0] ? o->m2l_share8 : -1;
        if (max_entries >= 3) out[2] = o->side[0] ? o->leaf_late : -1;
        if (max_entries >= 4) out[3] = o->side[0] ? o->near_split : -1;
        return MLFMA_OK;
    }
    return fail(MLFMA_EINVAL, "ops_variants: kernel %d has no variants", kernel);
}

int mlfma_ops_set_variant(mlfma_ops_t o, int kernel, int level, int variant)
{
    if (!o) return fail(MLFMA_EINVAL, "ops_set_variant: ops is NULL");
    if (kernel == MLFMA_K_M2L) {
        if (level < 3 || level > o->n_lev) return fail(MLFMA_EINVAL, "ops_set_variant: bad level %d", level);
        if (variant < 0 || variant > 9) return fail(MLFMA_EINVAL, "ops_set_variant: bad variant %d", variant);
        if (o->sampled && !sampled_m2l_form(variant))
            return fail(MLFMA_EINVAL, "ops_set_variant: M2L form %d needs full operator tables",
                        variant);
        o->lev[level].m2l_variant = variant;
    } else if (kernel == MLFMA_K_INTERP || kernel == MLFMA_K_ANTERP) {
        if (level < 3 || level >= o->n_lev)
            return fail(MLFMA_EINVAL, "ops_set_variant: bad level pair %d", level);
        const int nsh = dev::pair_onepass_shapes(o->lev[level + 1].L, o->lev[level].L);
        if (variant == kPairVariant) {
            if (!o->lev[level].pair_ok[kernel == MLFMA_K_INTERP ? 0 : 1])
                return fail(MLFMA_EINVAL, "ops_set_variant: pair kernel unavailable on level pair %d",
                            level);
        } else {
            if (variant < 0 || variant > std::max(1, nsh))
                return fail(MLFMA_EINVAL, "ops_set_variant: bad variant %d", variant);
            if (variant >= 1 && (!o->lev[level].onepass_ok || (o->flags & MLFMA_BF16X3_INTERP)))
                return fail(MLFMA_EINVAL,
                            "ops_set_variant: one-pass kernel unavailable on level pair %d", level);
        }
        (kernel == MLFMA_K_INTERP ? o->lev[level].interp_variant : o->lev[level].anterp_variant) =
            variant;
    } else if (kernel == MLFMA_K_P2P) {
        if (!o->side[0]) return fail(MLFMA_EINVAL, "ops_set_variant: one-stream handle has no schedule");
        if (level == 1) {
            if (variant < 1 || variant > 8) return fail(MLFMA_EINVAL, "ops_set_variant: bad M2L share %d", variant);
            o->m2l_share8 = variant;
        } else if (level == 2) {
            if (variant < 0 || variant > 1) return fail(MLFMA_EINVAL, "ops_set_variant: bad leaf M2L order %d", variant);
            o->leaf_late = variant;
        } else if (level == 3) {
            if (variant < 0 || variant > 1) return fail(MLFMA_EINVAL, "ops_set_variant: bad near-field split %d", variant);
            o->near_split = variant;
        } else {
            // fork points 3 and 4 need that many M2Ms in the upward pass
            if (variant < 0 || variant > 2 + std::min(2, std::max(0, o->n_lev - 3)))
                return fail(MLFMA_EINVAL, "ops_set_variant: bad variant %d", variant);
            o->near_fork = variant;
        }
    } else {
        return fail(MLFMA_EINVAL, "ops_set_variant: kernel %d has no variants", kernel);
    }
    free_graphs(o);  // captured graphs hold the old variant
    return MLFMA_OK;
}

int mlfma_profile_begin(mlfma_ops_t o, uint32_t kernel_mask, int64_t max_launches)
{
    if (!o) return fail(MLFMA_EINVAL, "profile_begin: ops is NULL");
    if (max_launches < 0 || max_launches > (1 << 20))
        return fail(MLFMA_EINVAL, "profile_begin: max_launches outside 0..2^20");
    prof_release(o, kProfPoolKeep);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(MLFMA_EDEVICE, "hipGetDevice failed");
    (void)hipSetDevice(o->device);
    int rc = MLFMA_OK;
    // grow the pool (timing only: no system-scope fence at their records,
    // which would write back caches in the middle of the timed work)
    while ((int64_t)o->prof_ev.size() < 2 * max_launches) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            rc = fail(MLFMA_EDEVICE, "profile_begin: hipEventCreate failed");
            break;
        }
        o->prof_ev.push_back(e);
    }
    (void)hipSetDevice(cur);
    if (rc) {
        prof_release(o);
        return rc;
    }
    o->prof_id.assign(max_launches, -1);
    o->prof_cap = max_launches;
    o->prof_used = 0;
    o->prof_mask = kernel_mask;
    return MLFMA_OK;
}

int mlfma_profile_end(mlfma_ops_t o, double *ms, int64_t *launches)
{
    if (!o || !ms || !launches) return fail(MLFMA_EINVAL, "profile_end: null argument");
    for (int i = 0; i < MLFMA_K_COUNT; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    int rc = MLFMA_OK;
    for (int64_t u = 0; u < o->prof_used; ++u) {
        float t = 0.f;
        if (hipEventSynchronize(o->prof_ev[2 * u + 1]) != hipSuccess ||
            hipEventElapsedTime(&t, o->prof_ev[2 * u], o->prof_ev[2 * u + 1]) != hipSuccess) {
            rc = fail(MLFMA_EDEVICE, "profile_end: event query failed");
            break;
        }
        ms[o->prof_id[u]] += t;
        launches[o->prof_id[u]] += 1;
    }
    prof_release(o, kProfPoolKeep);
    return rc;
}

int mlfma_ops_memory(mlfma_ops_t o, int64_t *operator_bytes, int64_t *total_bytes)
{
    if (!o) return fail(MLFMA_EINVAL, "ops_memory: ops is NULL");
    if (operator_bytes) *operator_bytes = o->operator_bytes;
    if (total_bytes) *total_bytes = o->planned_bytes;
    return MLFMA_OK;
}

const char *mlfma_status_string(int status)
{
    switch (status) {
    case MLFMA_OK: return "MLFMA_OK";
    case MLFMA_EINVAL: return "MLFMA_EINVAL: invalid argument";
    case MLFMA_EDEPTH: return "MLFMA_EDEPTH: tree too deep";
    case MLFMA_ENOMEM: return "MLFMA_ENOMEM: out of memory";
    case MLFMA_EDEVICE: return "MLFMA_EDEVICE: HIP device error";
    case MLFMA_ERANGE: return "MLFMA_ERANGE: point left its box";
    default: return "unknown status";
    }
}

const char *mlfma_last_error(void) { return last_error_text(); }

}  // extern "C"
