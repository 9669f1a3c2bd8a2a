// C-ABI entry points of the MRA library: tree upload, execution plan,
// memory sizing and the per-level launch schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mra.h"
#include "mra_internal.h"
#include "mra_kernels.h"

namespace mra {
int chain_lmax(int P);
hipError_t launch_chain(const KArgs& a, int mode, int grid, hipStream_t st);
hipError_t launch_prior_finish(const KArgs& a, int grid, hipStream_t st);
hipError_t launch_leaf(const KArgs& a, int grid, hipStream_t st);
hipError_t launch_small(const KArgs& a, int nmax, int mode, int grid, hipStream_t st);
hipError_t launch_fold_factor(const KArgs& a, int grid, hipStream_t st);
hipError_t launch_fold_gram(const KArgs& a, int grid, hipStream_t st);
hipError_t launch_final(const KArgs& a, int64_t nreg, int root_gram, hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st);
}  // namespace mra

using namespace mra;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// Largest observation count a region may hold and still fold in observation
// space (its scratch matrix is that count squared).  MRA_FACTOR_FOLD_MAX in
// the environment overrides the default (for tuning).
int64_t factor_fold_max() {
    const char* e = std::getenv("MRA_FACTOR_FOLD_MAX");
    if (e && *e) return std::max<int64_t>(0, std::atoll(e));
    return 192;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

template <class T>
int upload(T** dst, const std::vector<T>& v) {
    *dst = nullptr;
    const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (hipMalloc(reinterpret_cast<void**>(dst), bytes) != hipSuccess) return MRA_ENOMEM;
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return MRA_EDEVICE;
    return MRA_OK;
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice;
}

}  // namespace

struct mra_tree {
    HostTree h;
    int device = 0;
    uint32_t flags = 0;
    // device copies
    double *d_x = nullptr, *d_y = nullptr, *d_z = nullptr, *d_box = nullptr;
    int64_t *d_obs_lo = nullptr, *d_obs_hi = nullptr, *d_vst_off = nullptr, *d_gram_off = nullptr;
    int8_t* d_form = nullptr;
    // plan
    std::vector<int8_t> form;
    std::vector<int64_t> vst_off, gram_off;
    int64_t vst_size = 0, gram_size = 0;
    int WF = 1, WFs = 2;
    std::vector<std::vector<int>> prior_tasks, factor_tasks, gram_tasks;  // index by level (1..M-1)
    std::vector<int> leaf_tasks;                     // leaves with > 64 observations
    std::vector<int> small_tasks[3];                 // leaves with <= 16, 17..32, 33..64 observations
    std::vector<std::vector<int>> fsmall_tasks[3];   // factor folds with <= 16, 17..32, 33..64 rows, by level
    std::vector<int*> d_prior, d_factor, d_gramt, d_fsmall[3];
    int* d_leaf = nullptr;
    int* d_small[3] = {nullptr, nullptr, nullptr};
    int64_t scratch_leaf = 0, scratch_fold = 0;  // doubles per workgroup slot
    int root_gram = 0;
    int64_t n_gram = 0, leaf_min = 0, leaf_max = 0;
    // algorithmic FP64 flops of one theta, per launch kind and level
    std::vector<double> fl_chain, fl_pfin, fl_factor, fl_gram;
    double fl_leaf = 0.0, fl_small[3] = {0.0, 0.0, 0.0};
    std::vector<double> fl_fsmall[3];
    void* ws = nullptr;  // Workspace*, owned

    ~mra_tree();
    void free_device() {
        void* ps[] = {d_x, d_y, d_z, d_box, d_obs_lo, d_obs_hi, d_vst_off, d_gram_off, d_form, d_leaf,
                      d_small[0], d_small[1], d_small[2]};
        for (void* p : ps) if (p) (void)hipFree(p);
        for (auto* v : {&d_prior, &d_factor, &d_gramt, &d_fsmall[0], &d_fsmall[1], &d_fsmall[2]})
            for (int* p : *v) if (p) (void)hipFree(p);
    }
};

// Algorithmic FP64 flop counts of what each launch computes for one theta,
// with p = r_hat (padding excluded), n = observations of a region:
//   chain, level m knots : r_hat p^2 (m-1)^2  (per ancestor level l: the
//                          2 p^2 (l-1) product with earlier blocks and the
//                          p^2 triangular product with L_{A_l}^{-1})
//   chain, observations  : n p^2 (M-1)^2 summed over level-(M-1) regions
//   prior finish, m      : (m-1) p^3 + p^3/3 + p^3/3 (SYRK, Cholesky, inverse)
//   leaf finish          : (M-1) n^2 p + n^3/3 + n^2 ((M-1) p + 1)
//   factor fold, m       : n^2 p + n^3/3 + n^2 ((m-1) p + 1)
//   Gram fold, m         : sum_children n_c D^2 + p^3/3 + (D-p) p^2 + (D-p)^2 p,
//                          D = m p + 1 (Gram-form children: D^2/2 additions)
static void plan_flops(mra_tree& t) {
    const HostTree& h = t.h;
    const int M = h.M;
    const double p = h.rhat;
    t.fl_chain.assign(M + 1, 0.0);
    t.fl_pfin.assign(M, 0.0);
    t.fl_factor.assign(M, 0.0);
    t.fl_gram.assign(M, 0.0);
    for (int q = 0; q < 3; ++q) t.fl_fsmall[q].assign(M, 0.0);
    for (int m = 1; m < M; ++m) {
        const double nr = double(t.prior_tasks[m].size());
        t.fl_chain[m] = nr * p * p * p * double(m - 1) * (m - 1);
        t.fl_pfin[m] = nr * p * p * p * (double(m - 1) + 2.0 / 3.0);
        auto ff = [&](int g) {
            const double n = double(h.obs_hi[g] - h.obs_lo[g]);
            return n * n * p + n * n * n / 3.0 + n * n * ((m - 1) * p + 1);
        };
        for (int g : t.factor_tasks[m]) t.fl_factor[m] += ff(g);
        for (int q = 0; q < 3; ++q)
            for (int g : t.fsmall_tasks[q][m]) t.fl_fsmall[q][m] += ff(g);
        const double D = m * p + 1;
        for (int g : t.gram_tasks[m]) {
            const int64_t k = g - h.lvl_start[m - 1];
            double f = p * p * p / 3.0 + (D - p) * p * p + (D - p) * (D - p) * p;
            for (int j = 0; j < h.J; ++j) {
                const int64_t gc = h.lvl_start[m] + h.J * k + j;
                const double nc = double(h.obs_hi[gc] - h.obs_lo[gc]);
                if (m + 1 == M || t.form[gc] == FOLD_FACTOR) f += nc * D * D;
                else f += D * D / 2;
            }
            t.fl_gram[m] += f;
        }
    }
    const double L = M - 1;
    t.fl_chain[M] = double(h.n_used) * p * p * L * L;
    auto fl = [&](int g) {
        const double n = double(h.obs_hi[g] - h.obs_lo[g]);
        return L * n * n * p + n * n * n / 3.0 + n * n * (L * p + 1);
    };
    t.fl_leaf = t.fl_small[0] = t.fl_small[1] = t.fl_small[2] = 0.0;
    for (int g : t.leaf_tasks) t.fl_leaf += fl(g);
    for (int q = 0; q < 3; ++q)
        for (int g : t.small_tasks[q]) t.fl_small[q] += fl(g);
}

// ---- optional per-launch timing (HIP events around every launch) ----------
namespace {
struct ProfRec {
    int kind, level;
    hipEvent_t a, b;
    double flops;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
int g_prof_kind = -1, g_prof_level = -1;  // restrict to one (kernel, level); -1: all
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;  // events are created once and reused

hipEvent_t pooled_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
const char* const KIND_NAMES[] = {"k_chain", "k_prior_finish", "k_leaf_finish", "k_fold_factor", "k_fold_gram",
                                  "k_final", "k_small_leaf", "k_small_fold"};
}  // namespace

template <class F>
static hipError_t timed(int kind, int level, double flops, hipStream_t st, F&& launch) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on && (g_prof_kind < 0 || (g_prof_kind == kind && g_prof_level == level));
    }
    if (!on) return launch();
    ProfRec r{kind, level, nullptr, nullptr, flops};
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        r.a = pooled_event();
        r.b = pooled_event();
    }
    if (!r.a || !r.b) return launch();
    (void)hipEventRecord(r.a, st);
    const hipError_t e = launch();
    (void)hipEventRecord(r.b, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(r);
    return e;
}

extern "C" int mra_profile_enable(int on, const char* only_kernel, int only_level) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    g_prof_kind = -1;
    g_prof_level = -1;
    if (only_kernel) {
        for (int k = 0; k < int(sizeof(KIND_NAMES) / sizeof(KIND_NAMES[0])); ++k)
            if (std::strcmp(only_kernel, KIND_NAMES[k]) == 0) g_prof_kind = k;
        if (g_prof_kind < 0) return fail(MRA_EINVAL, std::string("unknown kernel name ") + only_kernel);
        g_prof_level = only_level;
    }
    return MRA_OK;
}

extern "C" int mra_profile_read(mra_kernel_stat* out, int cap, int* count) {
    if (!count) return fail(MRA_EINVAL, "count is NULL");
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        recs.swap(g_prof);
    }
    std::vector<mra_kernel_stat> agg;
    for (ProfRec& r : recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess) (void)hipEventElapsedTime(&ms, r.a, r.b);
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_event_pool.push_back(r.a);
            g_event_pool.push_back(r.b);
        }
        mra_kernel_stat* s = nullptr;
        for (auto& x : agg)
            if (x.level == r.level && std::strcmp(x.name, KIND_NAMES[r.kind]) == 0) s = &x;
        if (!s) {
            agg.push_back(mra_kernel_stat{});
            s = &agg.back();
            std::snprintf(s->name, sizeof s->name, "%s", KIND_NAMES[r.kind]);
            s->level = r.level;
        }
        s->launches += 1;
        s->ms += ms;
        s->flops += r.flops;
    }
    *count = int(agg.size());
    for (int i = 0; i < int(agg.size()) && i < cap; ++i) out[i] = agg[i];
    return MRA_OK;
}

extern "C" const char* mra_last_error(void) { return g_err.c_str(); }

extern "C" void mra_free_tree(mra_tree* t) { delete t; }

static int check_device() {
    int dev = 0, cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt == 0) {
        (void)hipGetLastError();
        return fail(MRA_EDEVICE, "no HIP device");
    }
    if (hipGetDevice(&dev) != hipSuccess) return fail(MRA_EDEVICE, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(MRA_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MRA_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    return MRA_OK;
}

extern "C" int mra_build_tree(const double* x, const double* y, const double* z, int64_t n, int J, int r, int M,
                              double offset, uint32_t flags, const double* domain4, mra_tree** out) {
    if (!out) return fail(MRA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n > 0 && (!x || !y || !z)) return fail(MRA_EINVAL, "x, y, z must not be NULL");
    if (n > (int64_t(1) << 31) - 1) return fail(MRA_EINVAL, "n must fit in 31 bits");
    int rc = check_device();
    if (rc) return rc;
    std::vector<double> hx, hy, hz;
    const double *px = x, *py = y, *pz = z;
    if (flags & MRA_DEVICE_PTRS) {
        hx.resize(n); hy.resize(n); hz.resize(n);
        if (n > 0 && (hipMemcpy(hx.data(), x, n * 8, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(hy.data(), y, n * 8, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(hz.data(), z, n * 8, hipMemcpyDeviceToHost) != hipSuccess))
            return fail(MRA_EDEVICE, "copy of device inputs failed");
        px = hx.data(); py = hy.data(); pz = hz.data();
    }
    auto* t = new mra_tree();
    t->flags = flags;
    (void)hipGetDevice(&t->device);
    std::string err;
    rc = build_host_tree(px, py, pz, n, J, r, M, offset, domain4, t->h, err);
    if (rc) { delete t; return fail(rc, err); }
    const HostTree& h = t->h;
    const int P = h.P;
    if (M - 1 > chain_lmax(P)) {
        delete t;
        return fail(MRA_EINVAL, "M - 1 = " + std::to_string(M - 1) + " exceeds " + std::to_string(chain_lmax(P)) +
                                    " levels above the finest for r_hat padded to " + std::to_string(P));
    }

    // plan: fold form of every non-leaf region, storage offsets, task lists
    t->form.assign(h.nreg, FOLD_FACTOR);
    t->vst_off.assign(h.nreg, -1);
    t->gram_off.assign(h.nreg, -1);
    t->prior_tasks.assign(M, {});
    t->factor_tasks.assign(M, {});
    t->gram_tasks.assign(M, {});
    for (int q = 0; q < 3; ++q) t->fsmall_tasks[q].assign(M, {});
    int64_t vo = 0, go = 0;
    for (int m = 1; m < M; ++m) {
        const int64_t thr = (flags & MRA_FOLD_GRAM) ? 0
                            : (flags & MRA_FOLD_FACTOR) ? 4096
                            : std::min<int64_t>(int64_t(m - 1) * P + 1, factor_fold_max());
        const int64_t D = int64_t(m) * P + 1;
        for (int64_t g = h.lvl_start[m - 1]; g < h.lvl_start[m]; ++g) {
            const int64_t np = h.obs_hi[g] - h.obs_lo[g];
            if (np == 0) continue;  // empty subtree: contributes nothing
            t->prior_tasks[m].push_back(int(g));
            t->vst_off[g] = vo;
            vo += int64_t(m) * P * P;
            if (np <= thr) {
                t->form[g] = FOLD_FACTOR;
                if (np <= 16) t->fsmall_tasks[0][m].push_back(int(g));
                else if (np <= 32) t->fsmall_tasks[1][m].push_back(int(g));
                else if (np <= 64) t->fsmall_tasks[2][m].push_back(int(g));
                else t->factor_tasks[m].push_back(int(g));
                if (np > 64) t->scratch_fold = std::max(t->scratch_fold, np * np);
            } else {
                t->form[g] = FOLD_GRAM;
                t->gram_tasks[m].push_back(int(g));
                t->gram_off[g] = go;
                go += D * D;
                ++t->n_gram;
            }
        }
    }
    t->vst_size = std::max<int64_t>(vo, 1);
    t->gram_size = std::max<int64_t>(go, 1);
    t->leaf_min = INT64_MAX;
    for (int64_t g = h.lvl_start[M - 1]; g < h.lvl_start[M]; ++g) {
        const int64_t nc = h.obs_hi[g] - h.obs_lo[g];
        t->leaf_min = std::min(t->leaf_min, nc);
        t->leaf_max = std::max(t->leaf_max, nc);
        if (nc > 64) {
            t->leaf_tasks.push_back(int(g));
            t->scratch_leaf = std::max(t->scratch_leaf, nc * nc);
        } else if (nc > 32) {
            t->small_tasks[2].push_back(int(g));
        } else if (nc > 16) {
            t->small_tasks[1].push_back(int(g));
        } else if (nc > 0) {
            t->small_tasks[0].push_back(int(g));
        }
    }
    if (t->leaf_min == INT64_MAX) t->leaf_min = 0;
    t->WF = (M - 1) * P + 1;
    t->WFs = (t->WF + 3) & ~3;
    t->root_gram = (M > 1 && t->form[0] == FOLD_GRAM) ? 1 : 0;
    plan_flops(*t);

    // device copies
    std::vector<int64_t> lo(h.obs_lo), hi(h.obs_hi);
    if ((rc = upload(&t->d_x, h.x)) || (rc = upload(&t->d_y, h.y)) || (rc = upload(&t->d_z, h.z)) ||
        (rc = upload(&t->d_box, h.box)) || (rc = upload(&t->d_obs_lo, lo)) || (rc = upload(&t->d_obs_hi, hi)) ||
        (rc = upload(&t->d_vst_off, t->vst_off)) || (rc = upload(&t->d_gram_off, t->gram_off)) ||
        (rc = upload(&t->d_form, t->form)) || (rc = upload(&t->d_leaf, t->leaf_tasks)) ||
        (rc = upload(&t->d_small[0], t->small_tasks[0])) || (rc = upload(&t->d_small[1], t->small_tasks[1])) ||
        (rc = upload(&t->d_small[2], t->small_tasks[2]))) {
        delete t;
        return fail(rc, "device allocation or copy failed while uploading the tree");
    }
    t->d_prior.assign(M, nullptr);
    t->d_factor.assign(M, nullptr);
    t->d_gramt.assign(M, nullptr);
    for (int q = 0; q < 3; ++q) t->d_fsmall[q].assign(M, nullptr);
    for (int m = 1; m < M; ++m)
        if ((rc = upload(&t->d_prior[m], t->prior_tasks[m])) || (rc = upload(&t->d_factor[m], t->factor_tasks[m])) ||
            (rc = upload(&t->d_gramt[m], t->gram_tasks[m])) || (rc = upload(&t->d_fsmall[0][m], t->fsmall_tasks[0][m])) ||
            (rc = upload(&t->d_fsmall[1][m], t->fsmall_tasks[1][m])) ||
            (rc = upload(&t->d_fsmall[2][m], t->fsmall_tasks[2][m]))) {
            delete t;
            return fail(rc, "device allocation failed for task lists");
        }
    *out = t;
    return MRA_OK;
}

extern "C" int mra_tree_info(const mra_tree* t, mra_info* info) {
    if (!t || !info) return fail(MRA_EINVAL, "NULL argument");
    const HostTree& h = t->h;
    info->n_in = h.n_in; info->n_nan = h.n_nan; info->n_elim = h.n_elim; info->n_used = h.n_used;
    info->J = h.J; info->M = h.M; info->r = h.r; info->r_hat = h.rhat; info->P = h.P;
    info->n_regions = h.nreg; info->n_leaves = h.nleaf;
    info->leaf_min = t->leaf_min; info->leaf_max = t->leaf_max;
    info->n_gram_regions = t->n_gram;
    return MRA_OK;
}

extern "C" int mra_tree_arrays(const mra_tree* t, double* x, double* y, double* z, int64_t* orig,
                               int64_t* leaf_off) {
    if (!t) return fail(MRA_EINVAL, "NULL tree");
    const HostTree& h = t->h;
    const size_t n = size_t(h.n_used);
    if (x) std::memcpy(x, h.x.data(), n * 8);
    if (y) std::memcpy(y, h.y.data(), n * 8);
    if (z) std::memcpy(z, h.z.data(), n * 8);
    if (orig) std::memcpy(orig, h.orig.data(), n * 8);
    if (leaf_off) {
        const int64_t l0 = h.lvl_start[h.M - 1];
        for (int64_t k = 0; k < h.nleaf; ++k) leaf_off[k] = h.obs_lo[l0 + k];
        leaf_off[h.nleaf] = h.n_used;
    }
    return MRA_OK;
}

static int smooth_of(int family, double nu, int* smooth) {
    if (family == MRA_EXP) { *smooth = 0; return MRA_OK; }
    if (family == MRA_MATERN && nu == 0.5) { *smooth = 0; return MRA_OK; }
    if (family == MRA_MATERN && nu == 1.5) { *smooth = 1; return MRA_OK; }
    return fail(MRA_EINVAL, "family must be MRA_EXP or MRA_MATERN with nu 0.5 or 1.5");
}

static int region_level(const HostTree& h, int64_t g) {
    for (int m = 1; m <= h.M; ++m) if (g < h.lvl_start[m]) return m;
    return h.M;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) { rc = fail(MRA_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); goto done; } \
    } while (0)

// Device workspace of a tree, kept between calls (allocation of the large
// buffers is not repeated per evaluation).  Calls on one tree are serialised:
// a call on a different stream first waits for the previous call's work.
struct Workspace {
    double *vst = nullptr, *F = nullptr, *gram = nullptr, *dval = nullptr, *scratch = nullptr;
    double *th = nullptr, *out = nullptr;
    int* status = nullptr;
    int64_t Bc = 0, nslot = 0, scratch_per = 0, cap_B = 0;
    bool mem_limited = false;  // Bc was capped by device memory, not by the request
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    void release() {
        if (done) { (void)hipEventSynchronize(done); (void)hipEventDestroy(done); done = nullptr; }
        for (void* p : {static_cast<void*>(vst), static_cast<void*>(F), static_cast<void*>(gram),
                        static_cast<void*>(dval), static_cast<void*>(scratch), static_cast<void*>(th),
                        static_cast<void*>(out), static_cast<void*>(status)})
            if (p) (void)hipFree(p);
        vst = F = gram = dval = scratch = th = out = nullptr;
        status = nullptr;
        Bc = nslot = cap_B = 0;
        used = false;
    }
};

static std::mutex g_ws_mu;

static Workspace& workspace_of(const mra_tree* t);

static int ensure_workspace(const mra_tree* t, Workspace& w, int64_t B, hipStream_t st) {
    const HostTree& h = t->h;
    const int64_t F_stride = std::max<int64_t>(h.n_used, 1) * t->WFs;
    const int64_t per_theta = t->vst_size + F_stride + t->gram_size + h.nreg;
    const int64_t scratch_per = std::max<int64_t>({t->scratch_leaf, t->scratch_fold, 1});
    // reuse when the buffers hold enough theta per chunk (or could not hold more)
    if (w.Bc > 0 && w.cap_B >= B && (w.Bc >= B || w.mem_limited)) return MRA_OK;
    if (w.Bc > 0) {
        // grow: wait for the last user, release, reallocate
        w.release();
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(MRA_EDEVICE, "hipMemGetInfo failed");
    const double budget = 0.6 * double(free_b) / 8.0;  // doubles
    const int64_t nslot = std::min<int64_t>(2048, std::max<int64_t>(1, int64_t(0.2 * budget / double(scratch_per))));
    const double left = budget - double(nslot) * double(scratch_per);
    const int64_t Bc = std::min<int64_t>(std::max<int64_t>(B, 1), int64_t(left / double(per_theta)));
    if (Bc < 1) return fail(MRA_ENOMEM, "not enough device memory for one theta");
    const int64_t capB = std::max<int64_t>(B, 64);
    auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 8)) == hipSuccess; };
    if (!al(reinterpret_cast<void**>(&w.vst), size_t(Bc) * t->vst_size * 8) ||
        !al(reinterpret_cast<void**>(&w.F), size_t(Bc) * F_stride * 8) ||
        !al(reinterpret_cast<void**>(&w.gram), size_t(Bc) * t->gram_size * 8) ||
        !al(reinterpret_cast<void**>(&w.dval), size_t(Bc) * h.nreg * 8) ||
        !al(reinterpret_cast<void**>(&w.scratch), size_t(nslot) * scratch_per * 8) ||
        !al(reinterpret_cast<void**>(&w.status), size_t(capB) * sizeof(int)) ||
        !al(reinterpret_cast<void**>(&w.th), size_t(capB) * 3 * 8) ||
        !al(reinterpret_cast<void**>(&w.out), size_t(capB) * 8)) {
        (void)hipGetLastError();
        w.release();
        return fail(MRA_ENOMEM, "device allocation of the evaluation workspace failed");
    }
    if (hipEventCreateWithFlags(&w.done, hipEventDisableTiming) != hipSuccess) {
        w.release();
        return fail(MRA_EDEVICE, "hipEventCreate failed");
    }
    w.Bc = Bc;
    w.mem_limited = Bc < std::max<int64_t>(B, 1);
    w.nslot = nslot;
    w.scratch_per = scratch_per;
    w.cap_B = capB;
    w.last = st;
    return MRA_OK;
}

extern "C" int mra_loglik(const mra_tree* t, int family, double nu, const double* theta, int64_t B,
                          double* loglik, void* stream) {
    if (!t || !theta || !loglik || B < 1) return fail(MRA_EINVAL, "NULL argument or B < 1");
    int smooth = 0;
    int rc = smooth_of(family, nu, &smooth);
    if (rc) return rc;
    const HostTree& h = t->h;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const bool dev = is_device_ptr(theta);
    if (dev != is_device_ptr(loglik)) return fail(MRA_EINVAL, "theta and loglik must be in the same memory space");
    if (!dev) {
        for (int64_t b = 0; b < B; ++b) {
            const double* q = theta + 3 * b;
            if (!(q[0] > 0.0) || !(q[1] > 0.0) || !(q[2] > 0.0) || !std::isfinite(q[0]) || !std::isfinite(q[1]) ||
                !std::isfinite(q[2]))
                return fail(MRA_EINVAL, "theta " + std::to_string(b) + ": alpha, beta, tau must be finite and > 0");
        }
    }
    const int M = h.M, P = h.P;
    const int64_t F_stride = std::max<int64_t>(h.n_used, 1) * t->WFs;

    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace& w = workspace_of(t);
    rc = ensure_workspace(t, w, B, st);
    if (rc) return rc;
    if (w.used && w.last != st) (void)hipStreamWaitEvent(st, w.done, 0);
    const int64_t Bc = w.Bc, nslot = w.nslot;
    double* d_th = dev ? const_cast<double*>(theta) : w.th;
    double* d_out = dev ? loglik : w.out;
    int* status = w.status;
    std::vector<int> hstatus;
    KArgs a{};
    if (!dev) HIPCHK(hipMemcpyAsync(d_th, theta, 3 * B * 8, hipMemcpyHostToDevice, st));
    HIPCHK(launch_fill_int(status, B, 0, st));

    a.x = t->d_x; a.y = t->d_y; a.z = t->d_z; a.box = t->d_box;
    a.obs_lo = t->d_obs_lo; a.obs_hi = t->d_obs_hi;
    a.vst_off = t->d_vst_off; a.gram_off = t->d_gram_off; a.form = t->d_form;
    for (int m = 0; m <= M && m <= MAXL; ++m) a.lvl[m] = h.lvl_start[m];
    a.J = h.J; a.M = M; a.nx = h.nx; a.ny = h.ny; a.rhat = h.rhat; a.P = P; a.WF = t->WF; a.WFs = t->WFs;
    a.offset = h.offset; a.smooth = smooth;
    a.vst = w.vst; a.vst_stride = t->vst_size;
    a.F = w.F; a.F_stride = F_stride;
    a.gram = w.gram; a.gram_stride = t->gram_size;
    a.dval = w.dval; a.d_stride = h.nreg;
    a.scratch = w.scratch; a.scratch_stride = w.scratch_per;
    a.n_used = double(h.n_used);

    for (int64_t b0 = 0; b0 < B; b0 += Bc) {
        const int nb = int(std::min<int64_t>(Bc, B - b0));
        a.theta = d_th + 3 * b0;
        a.ntheta = nb;
        a.status = status + b0;
        a.out = d_out + b0;
        HIPCHK(launch_fill(w.dval, int64_t(nb) * h.nreg, 0.0, st));
        for (int m = 1; m < M; ++m) {
            a.level = m;
            a.tasks = t->d_prior[m];
            a.ntasks = int64_t(t->prior_tasks[m].size());
            if (a.ntasks == 0) continue;
            const int grid = int(std::min<int64_t>(a.ntasks * nb, 1 << 16));
            if (m > 1) HIPCHK(timed(0, m, t->fl_chain[m] * nb, st, [&] { return launch_chain(a, 0, grid, st); }));
            HIPCHK(timed(1, m, t->fl_pfin[m] * nb, st, [&] { return launch_prior_finish(a, grid, st); }));
        }
        if (M > 1 && !t->prior_tasks[M - 1].empty()) {
            a.level = M - 1;
            a.tasks = t->d_prior[M - 1];
            a.ntasks = int64_t(t->prior_tasks[M - 1].size());
            const int grid = int(std::min<int64_t>(a.ntasks * nb, 1 << 16));
            HIPCHK(timed(0, M, t->fl_chain[M] * nb, st, [&] { return launch_chain(a, 1, grid, st); }));
        }
        a.level = M;
        for (int q = 0; q < 3; ++q) {
            a.tasks = t->d_small[q];
            a.ntasks = int64_t(t->small_tasks[q].size());
            if (a.ntasks > 0)
                HIPCHK(timed(6, M, t->fl_small[q] * nb, st, [&] {
                    return launch_small(a, 16 << q, 0, int(std::min<int64_t>(a.ntasks * nb, 1 << 18)), st);
                }));
        }
        a.tasks = t->d_leaf;
        a.ntasks = int64_t(t->leaf_tasks.size());
        if (a.ntasks > 0)
            HIPCHK(timed(2, M, t->fl_leaf * nb, st, [&] { return launch_leaf(a, int(std::min<int64_t>(a.ntasks * nb, nslot)), st); }));
        for (int m = M - 1; m >= 1; --m) {
            a.level = m;
            for (int q = 0; q < 3; ++q) {
                a.tasks = t->d_fsmall[q][m];
                a.ntasks = int64_t(t->fsmall_tasks[q][m].size());
                if (a.ntasks > 0)
                    HIPCHK(timed(7, m, t->fl_fsmall[q][m] * nb, st, [&] {
                        return launch_small(a, 16 << q, 1, int(std::min<int64_t>(a.ntasks * nb, 1 << 18)), st);
                    }));
            }
            a.tasks = t->d_factor[m];
            a.ntasks = int64_t(t->factor_tasks[m].size());
            if (a.ntasks > 0)
                HIPCHK(timed(3, m, t->fl_factor[m] * nb, st, [&] { return launch_fold_factor(a, int(std::min<int64_t>(a.ntasks * nb, nslot)), st); }));
            a.tasks = t->d_gramt[m];
            a.ntasks = int64_t(t->gram_tasks[m].size());
            if (a.ntasks > 0)
                HIPCHK(timed(4, m, t->fl_gram[m] * nb, st, [&] { return launch_fold_gram(a, int(std::min<int64_t>(a.ntasks * nb, 1 << 16)), st); }));
        }
        HIPCHK(timed(5, 0, 0.0, st, [&] { return launch_final(a, h.nreg, t->root_gram, st); }));
    }
    (void)hipEventRecord(w.done, st);
    w.last = st;
    w.used = true;
    if (!dev) {
        HIPCHK(hipMemcpyAsync(loglik, d_out, B * 8, hipMemcpyDeviceToHost, st));
        hstatus.resize(B);
        HIPCHK(hipMemcpyAsync(hstatus.data(), status, B * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int64_t b = 0; b < B; ++b)
            if (hstatus[b] != 0) {
                const int64_t g = hstatus[b] - 1;
                const int lev = region_level(h, g);
                rc = fail(MRA_ENOTPD, "not positive definite: theta " + std::to_string(b) + ", level " +
                                          std::to_string(lev) + ", region " + std::to_string(g - h.lvl_start[lev - 1]));
                break;
            }
    }
done:
    return rc;
}

static Workspace& workspace_of(const mra_tree* t) {
    auto* mt = const_cast<mra_tree*>(t);
    if (!mt->ws) mt->ws = new Workspace();
    return *static_cast<Workspace*>(mt->ws);
}

mra_tree::~mra_tree() {
    if (ws) {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        static_cast<Workspace*>(ws)->release();
        delete static_cast<Workspace*>(ws);
    }
    free_device();
}

extern "C" int mra_predict(const mra_tree* t, int family, double nu, const double* theta, const double* px,
                           const double* py, int64_t np, double* mean, double* var, void* stream) {
    (void)t; (void)family; (void)nu; (void)theta; (void)px; (void)py; (void)np; (void)mean; (void)var;
    (void)stream;
    return fail(MRA_EINVAL, "mra_predict is not available in this build yet");
}
