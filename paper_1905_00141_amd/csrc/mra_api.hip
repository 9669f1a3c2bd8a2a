// C-ABI entry points of the MRA library: tree upload, execution plans,
// device workspace, the per-level launch schedule, graph capture of repeated
// evaluations, and kriging.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
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
hipError_t launch_gram_panel(const KArgs& a, int grid, hipStream_t st);
hipError_t launch_gram_tile(const KArgs& a, hipStream_t st);
hipError_t launch_gram_tile2(const KArgs& a, hipStream_t st);
hipError_t launch_final(const KArgs& a, int64_t nreg, int root_gram, hipStream_t st);
hipError_t launch_pred_leaf(const KArgs& a, int grid, hipStream_t st);
hipError_t launch_pred_fold(const KArgs& a, hipStream_t st);
hipError_t launch_pred_out(const KArgs& a, hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st);
hipError_t launch_rep(const double* theta, int nb, int* rep, hipStream_t st);
hipError_t launch_rep_status(const int* rep, int nb, int* status, hipStream_t st);
}  // namespace mra

namespace mra {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
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

int check_device() {
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

}  // namespace mra

using namespace mra;

namespace {

// Largest observation count a region may hold and still fold in observation
// space (its scratch matrix is that count squared).  MRA_FACTOR_FOLD_MAX in
// the environment overrides the default (for tuning).
int64_t factor_fold_max() {
    const char* e = std::getenv("MRA_FACTOR_FOLD_MAX");
    if (e && *e) return std::max<int64_t>(0, std::atoll(e));
    return 192;
}

template <class T>
int upload(T** dst, const std::vector<T>& v) {
    *dst = nullptr;
    const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (hipMalloc(reinterpret_cast<void**>(dst), bytes) != hipSuccess) return MRA_ENOMEM;
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return MRA_EDEVICE;
    return MRA_OK;
}

int64_t ipow_h(int64_t b, int e) {
    int64_t v = 1;
    while (e-- > 0) v *= b;
    return v;
}

}  // namespace

// Execution plan over a tree: which regions take part, how each folds
// (observation space for few observations, knot space otherwise), storage
// offsets, per-level task lists (host and device) and the algorithmic flop
// counts of every launch.
struct Plan {
    std::vector<int8_t> form;
    std::vector<int64_t> vst_off, gram_off;
    int64_t vst_size = 1, gram_size = 1;
    std::vector<std::vector<int>> prior_tasks, factor_tasks, gram_tasks;  // by level 1..M-1
    std::vector<std::vector<int>> fsmall_tasks[3];  // factor folds with <= 16, 17..32, 33..64 rows
    std::vector<int> leaf_tasks;                    // leaves with > 64 observations
    std::vector<int> small_tasks[3];                // leaves with <= 16, 17..32, 33..64 observations
    std::vector<int> chain_obs_tasks;               // level-(M-1) regions with observations
    std::vector<int64_t> s0_off;                    // per leaf: offset of its C - V V^T (theta with a shared prior)
    int64_t s0_size = 1;
    int64_t scratch_leaf = 0, scratch_fold = 0;     // doubles per workgroup slot
    int root_gram = 0;
    int64_t n_gram = 0;
    // device copies
    int8_t* d_form = nullptr;
    int64_t *d_vst_off = nullptr, *d_gram_off = nullptr;
    std::vector<int*> d_prior, d_factor, d_gramt, d_fsmall[3];
    int *d_leaf = nullptr, *d_small[3] = {nullptr, nullptr, nullptr}, *d_chain_obs = nullptr;
    int64_t* d_s0_off = nullptr;
    // algorithmic FP64 flops of one theta
    std::vector<double> fl_chain, fl_pfin, fl_factor, fl_gram, fl_gtile, fl_fsmall[3];
    // knot-space blocks of level m staged through LDS in 128 x 128 super-blocks
    // (pays off when the regions' observation-space children hold many rows;
    // measured on config 3: 24 % faster at a median of 308 rows, 14 % slower
    // at a median of 0)
    std::vector<int8_t> gtile_super;
    double fl_chain_obs = 0.0, fl_leaf = 0.0, fl_small[3] = {0.0, 0.0, 0.0};
    // the part of fl_leaf / fl_small that forms C - V V^T: (M-1) n^2 p
    double fl_leaf_s = 0.0, fl_small_s[3] = {0.0, 0.0, 0.0};

    ~Plan() {
        void* ps[] = {d_form, d_vst_off, d_gram_off, d_leaf, d_small[0], d_small[1], d_small[2], d_chain_obs, d_s0_off};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        for (auto* v : {&d_prior, &d_factor, &d_gramt, &d_fsmall[0], &d_fsmall[1], &d_fsmall[2]})
            for (int* p : *v)
                if (p) (void)hipFree(p);
    }
};

// Execution choices that change which kernel handles a region, never the
// result beyond rounding: the largest subtree (observations) folded in
// observation space per level (-1: the default rule) and the largest leaf or
// fold handled by the one-wave finishers (16, 32 or 64).
struct PlanOpts {
    std::vector<int64_t> fold_max;  // index m = 1 .. M-1
    int small_max = 64;
    std::vector<int8_t> tile;       // index m: -1 default rule, 0 64 x 64 blocks, 1 128 x 128 super-blocks
};

struct mra_tree {
    HostTree h;
    PlanOpts opts;
    int device = 0;
    uint32_t flags = 0;
    double *d_x = nullptr, *d_y = nullptr, *d_z = nullptr, *d_box = nullptr;
    int64_t* d_orig = nullptr;  // input index of each grouped observation (GPU-built trees)
    int64_t *d_obs_lo = nullptr, *d_obs_hi = nullptr;
    int WF = 1, WFs = 4;
    int fa_cols = 0;  // further approximation: columns before column 0 of an F row (the leaf's own knots)
    Plan lik;  // plan of the likelihood
    int64_t leaf_min = 0, leaf_max = 0;
    int64_t leaf_hist[16] = {0};
    int64_t chunk_multiple = 1;  // theta per chunk rounded down to a multiple of this
    void* ws = nullptr;  // Workspace*, owned
    ~mra_tree();
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
//   Gram fold, m, panel  : 2 K D p + 2 K Dt + 2 p^3/3 + Dt p^2 + 2 Dt p
//   Gram fold, m, blocks : Ds (Ds + 1) (K + p)
//                          with K the rows of the region's observation-space
//                          children, D = m p + 1, Dt = D - p, Ds = (m-1) p
//                          (knot-space children contribute additions only)
// With the further approximation (fa) the leaves have a prior too (level M)
// and the observation rows one more level: chain n p^2 M^2, leaf matrix n^2 p.
static void plan_flops(const HostTree& h, Plan& t, bool fa) {
    const int M = h.M;
    const double p = h.rhat;
    t.fl_chain.assign(M + 1, 0.0);
    t.fl_pfin.assign(M + 1, 0.0);
    t.fl_factor.assign(M, 0.0);
    t.fl_gram.assign(M, 0.0);
    t.fl_gtile.assign(M, 0.0);
    t.gtile_super.assign(M, 0);
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
        const double D = m * p + 1, Dt = D - p, Ds = (m - 1) * p;
        std::vector<double> kfs;
        for (int g : t.gram_tasks[m]) {
            const int64_t k = g - h.lvl_start[m - 1];
            double kf = 0.0;  // rows of the observation-space children
            for (int j = 0; j < h.J; ++j) {
                const int64_t gc = h.lvl_start[m] + h.J * k + j;
                if (m + 1 == M || t.form[gc] == FOLD_FACTOR) kf += double(h.obs_hi[gc] - h.obs_lo[gc]);
            }
            // panel: first block column and data row of G, factor, inverse, Z, data row of S
            t.fl_gram[m] += 2 * kf * D * p + 2 * kf * Dt + p * p * p * (2.0 / 3.0) + Dt * p * p + 2 * Dt * p;
            // blocks of S below the data row (lower triangle): G part and Z Z^T
            t.fl_gtile[m] += Ds * (Ds + 1) * (kf + p);
            kfs.push_back(kf);
        }
        // super-blocks when the typical (median) region has >= 128 such rows
        if (!kfs.empty()) {
            std::nth_element(kfs.begin(), kfs.begin() + kfs.size() / 2, kfs.end());
            t.gtile_super[m] = kfs[kfs.size() / 2] >= 128.0;
        }
    }
    if (fa && M < int(t.prior_tasks.size())) {
        const double nr = double(t.prior_tasks[M].size());
        t.fl_chain[M] = nr * p * p * p * double(M - 1) * (M - 1);
        t.fl_pfin[M] = nr * p * p * p * (double(M - 1) + 2.0 / 3.0);
    }
    const double L = M - 1, Lc = fa ? M : M - 1, Ls = fa ? 1 : M - 1;
    t.fl_chain_obs = double(h.n_used) * p * p * Lc * Lc;
    auto fl = [&](int g) {
        const double n = double(h.obs_hi[g] - h.obs_lo[g]);
        return Ls * n * n * p + n * n * n / 3.0 + n * n * (L * p + 1);
    };
    auto fls = [&](int g) {
        const double n = double(h.obs_hi[g] - h.obs_lo[g]);
        return Ls * n * n * p;
    };
    t.fl_leaf = t.fl_leaf_s = 0.0;
    for (int g : t.leaf_tasks) t.fl_leaf += fl(g), t.fl_leaf_s += fls(g);
    for (int q = 0; q < 3; ++q) {
        t.fl_small[q] = t.fl_small_s[q] = 0.0;
        for (int g : t.small_tasks[q]) t.fl_small[q] += fl(g), t.fl_small_s[q] += fls(g);
    }
}

// Build a plan.  active[g] (optional) marks regions whose prior is needed
// beyond those holding observations (prediction points); gram_only forces
// every fold into knot space.
static int make_plan(const HostTree& h, uint32_t flags, bool gram_only, const std::vector<int64_t>* extra_count,
                     const PlanOpts* opts, Plan& t, std::string& err) {
    const int64_t smax = opts ? opts->small_max : 64;
    const int M = h.M, P = h.P;
    const bool fa = (flags & MRA_FURTHER_APPROX) != 0;
    t.form.assign(h.nreg, FOLD_FACTOR);
    t.vst_off.assign(h.nreg, -1);
    t.gram_off.assign(h.nreg, -1);
    t.prior_tasks.assign(M + 1, {});
    t.factor_tasks.assign(M, {});
    t.gram_tasks.assign(M, {});
    for (int q = 0; q < 3; ++q) t.fsmall_tasks[q].assign(M, {});
    int64_t vo = 0, go = 0;
    // fold form of every region, bottom-up: observation space when the
    // subtree holds at most the level's threshold AND every child above the
    // finest level that holds observations folds in observation space too
    // (an observation-space fold works on its rows' F columns, which only
    // observation-space descendants keep up to date)
    for (int m = M - 1; m >= 1; --m) {
        int64_t thr = (gram_only || (flags & MRA_FOLD_GRAM)) ? 0
                      : (flags & MRA_FOLD_FACTOR) ? 4096
                      : std::min<int64_t>(int64_t(m - 1) * P + 1, factor_fold_max());
        if (!gram_only && !(flags & (MRA_FOLD_GRAM | MRA_FOLD_FACTOR)) && opts && m < int64_t(opts->fold_max.size()) &&
            opts->fold_max[m] >= 0)
            thr = opts->fold_max[m];
        for (int64_t g = h.lvl_start[m - 1]; g < h.lvl_start[m]; ++g) {
            const int64_t np = h.obs_hi[g] - h.obs_lo[g];
            bool fac = np <= thr;
            if (fac && m + 1 < M)
                for (int j = 0; j < h.J; ++j) {
                    const int64_t gc = h.lvl_start[m] + (g - h.lvl_start[m - 1]) * h.J + j;
                    if (h.obs_hi[gc] > h.obs_lo[gc] && t.form[gc] != FOLD_FACTOR) fac = false;
                }
            t.form[g] = fac ? FOLD_FACTOR : FOLD_GRAM;
        }
    }
    for (int m = 1; m < M; ++m) {
        const int64_t D = int64_t(m) * P + 1;
        for (int64_t g = h.lvl_start[m - 1]; g < h.lvl_start[m]; ++g) {
            const int64_t np = h.obs_hi[g] - h.obs_lo[g];
            const int64_t ne = extra_count ? (*extra_count)[g] : 0;
            if (np == 0 && ne == 0) continue;  // nothing below: no prior, no fold
            t.prior_tasks[m].push_back(int(g));
            t.vst_off[g] = vo;
            vo += int64_t(m) * P * P;
            if (np == 0) continue;             // prior only (prediction points below)
            if (t.form[g] == FOLD_FACTOR) {
                if (np <= 16 && np <= smax) t.fsmall_tasks[0][m].push_back(int(g));
                else if (np <= 32 && np <= smax) t.fsmall_tasks[1][m].push_back(int(g));
                else if (np <= 64 && np <= smax) t.fsmall_tasks[2][m].push_back(int(g));
                else {
                    t.factor_tasks[m].push_back(int(g));
                    // the matrix, rows padded to a multiple of 4
                    t.scratch_fold = std::max(t.scratch_fold, np * ((np + 3) & ~int64_t(3)));
                }
            } else {
                t.gram_tasks[m].push_back(int(g));
                t.gram_off[g] = go;
                go += D * D;
                ++t.n_gram;
            }
        }
        if (m == M - 1 && !fa)
            for (int g : t.prior_tasks[m])
                if (h.obs_hi[g] > h.obs_lo[g]) t.chain_obs_tasks.push_back(g);
    }
    if (fa) {
        // the leaves' own knots: a prior (M blocks of V store each) for every
        // leaf with observations, and the observation rows tasked per leaf
        for (int64_t g = h.lvl_start[M - 1]; g < h.lvl_start[M]; ++g) {
            if (h.obs_hi[g] == h.obs_lo[g]) continue;
            t.prior_tasks[M].push_back(int(g));
            t.vst_off[g] = vo;
            vo += int64_t(M) * P * P;
            t.chain_obs_tasks.push_back(int(g));
        }
    }
    t.vst_size = std::max<int64_t>(vo, 1);
    t.gram_size = std::max<int64_t>(go, 1);
    t.s0_off.assign(size_t(h.lvl_start[M] - h.lvl_start[M - 1]), 0);
    int64_t s0 = 0;
    for (int64_t g = h.lvl_start[M - 1]; g < h.lvl_start[M]; ++g) {
        const int64_t nc = h.obs_hi[g] - h.obs_lo[g];
        t.s0_off[size_t(g - h.lvl_start[M - 1])] = s0;
        s0 += nc * ((nc + 3) & ~int64_t(3));
        if (nc > smax) {
            t.leaf_tasks.push_back(int(g));
            t.scratch_leaf = std::max(t.scratch_leaf, nc * ((nc + 3) & ~int64_t(3)));
        } else if (nc > 32) {
            t.small_tasks[2].push_back(int(g));
        } else if (nc > 16) {
            t.small_tasks[1].push_back(int(g));
        } else if (nc > 0) {
            t.small_tasks[0].push_back(int(g));
        }
    }
    // the workgroup finishers take their tasks largest first (longest
    // processing time first: the last tasks to start are the short ones)
    auto by_size = [&h](std::vector<int>& v) {
        std::stable_sort(v.begin(), v.end(), [&h](int p, int q) {
            return h.obs_hi[p] - h.obs_lo[p] > h.obs_hi[q] - h.obs_lo[q];
        });
    };
    by_size(t.leaf_tasks);
    for (int m = 1; m < M; ++m) by_size(t.factor_tasks[m]);
    t.s0_size = std::max<int64_t>((s0 + 31) & ~int64_t(31), 1);
    t.root_gram = (M > 1 && t.form[0] == FOLD_GRAM && t.gram_off[0] >= 0) ? 1 : 0;
    plan_flops(h, t, fa);
    if (opts)
        for (int m = 1; m < M && m < int(opts->tile.size()); ++m)
            if (opts->tile[m] >= 0) t.gtile_super[m] = opts->tile[m];
    int rc;
    if ((rc = upload(&t.d_vst_off, t.vst_off)) || (rc = upload(&t.d_gram_off, t.gram_off)) ||
        (rc = upload(&t.d_form, t.form)) || (rc = upload(&t.d_leaf, t.leaf_tasks)) ||
        (rc = upload(&t.d_small[0], t.small_tasks[0])) || (rc = upload(&t.d_small[1], t.small_tasks[1])) ||
        (rc = upload(&t.d_small[2], t.small_tasks[2])) || (rc = upload(&t.d_chain_obs, t.chain_obs_tasks)) ||
        (rc = upload(&t.d_s0_off, t.s0_off))) {
        err = "device allocation failed for the execution plan";
        return rc;
    }
    t.d_prior.assign(M + 1, nullptr);
    t.d_factor.assign(M, nullptr);
    t.d_gramt.assign(M, nullptr);
    for (int q = 0; q < 3; ++q) t.d_fsmall[q].assign(M, nullptr);
    if (fa && (rc = upload(&t.d_prior[M], t.prior_tasks[M]))) {
        err = "device allocation failed for the execution plan";
        return rc;
    }
    for (int m = 1; m < M; ++m)
        if ((rc = upload(&t.d_prior[m], t.prior_tasks[m])) || (rc = upload(&t.d_factor[m], t.factor_tasks[m])) ||
            (rc = upload(&t.d_gramt[m], t.gram_tasks[m])) || (rc = upload(&t.d_fsmall[0][m], t.fsmall_tasks[0][m])) ||
            (rc = upload(&t.d_fsmall[1][m], t.fsmall_tasks[1][m])) ||
            (rc = upload(&t.d_fsmall[2][m], t.fsmall_tasks[2][m]))) {
            err = "device allocation failed for the execution plan";
            return rc;
        }
    return MRA_OK;
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
const char* const KIND_NAMES[] = {"k_chain",     "k_prior_finish", "k_leaf_finish", "k_fold_factor",
                                  "k_gram_panel", "k_final",       "k_small_leaf",  "k_small_fold",
                                  "k_pred_leaf",  "k_pred_fold",   "k_gram_tile",  "k_gram_tile2"};
}  // namespace

// Set while an entry point that must not create HIP objects enqueues its
// launches (per-launch timing would create events).
thread_local bool t_untimed = false;

template <class F>
static hipError_t timed(int kind, int level, double flops, hipStream_t st, F&& launch) {
    if (t_untimed) return launch();
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

extern "C" int mra_build_tree(const double* x, const double* y, const double* z, int64_t n, int J, int r, int M,
                              double offset, uint32_t flags, const double* domain4, mra_tree** out) {
    if (!out) return fail(MRA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n > 0 && (!x || !y || !z)) return fail(MRA_EINVAL, "x, y, z must not be NULL");
    if (n > (int64_t(1) << 31) - 1) return fail(MRA_EINVAL, "n must fit in 31 bits");
    int rc = check_device();
    if (rc) return rc;
    // the partition is built on the GPU, except with duplicate elimination
    // (host build; MRA_HOST_TREE=1 in the environment also selects it)
    const char* ht = std::getenv("MRA_HOST_TREE");
    const bool on_gpu = !(flags & MRA_ELIM_DUPLICATES) && !(ht && *ht == '1');
    std::vector<double> hx, hy, hz;
    const double *px = x, *py = y, *pz = z;
    if ((flags & MRA_DEVICE_PTRS) && (!on_gpu || M <= 0)) {
        hx.resize(n); hy.resize(n); hz.resize(n);
        if (n > 0 && (hipMemcpy(hx.data(), x, n * 8, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(hy.data(), y, n * 8, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(hz.data(), z, n * 8, hipMemcpyDeviceToHost) != hipSuccess))
            return fail(MRA_EDEVICE, "copy of device inputs failed");
        px = hx.data(); py = hy.data(); pz = hz.data();
    }
    if (M <= 0) {
        // NUM_LEVELS_M "default" (Sec. 2.2): the finest level's average count
        // per region closest, on a log scale, to the knots per coarser region
        if (J != 2 && J != 4) return fail(MRA_EINVAL, "J must be 2 or 4");
        if (r < 1) return fail(MRA_EINVAL, "r must be >= 1");
        int64_t nobs = 0;
        for (int64_t i = 0; i < n; ++i) nobs += std::isnan(pz[i]) ? 0 : 1;
        int nx = 1;
        while (int64_t(nx) * nx < r) ++nx;
        const int64_t rhat = int64_t(nx) * (r / nx);
        M = 1;
        if (nobs > rhat) M = 1 + std::max(0, int(std::floor(std::log(double(nobs) / double(rhat)) / std::log(double(J)) + 0.5)));
    }
    auto* t = new mra_tree();
    t->flags = flags;
    (void)hipGetDevice(&t->device);
    std::string err;
    if (on_gpu) {
        // device inputs: the caller's (MRA_DEVICE_PTRS) or a temporary copy
        const double *dx = x, *dy = y, *dz = z;
        double* up[3] = {nullptr, nullptr, nullptr};
        if (!(flags & MRA_DEVICE_PTRS)) {
            const double* src[3] = {x, y, z};
            for (int c = 0; c < 3; ++c)
                if (hipMalloc(reinterpret_cast<void**>(&up[c]), std::max<int64_t>(n, 1) * 8) != hipSuccess ||
                    (n > 0 && hipMemcpy(up[c], src[c], n * 8, hipMemcpyHostToDevice) != hipSuccess)) {
                    for (double* p : up) if (p) (void)hipFree(p);
                    delete t;
                    return fail(MRA_ENOMEM, "device copy of the inputs failed");
                }
            dx = up[0]; dy = up[1]; dz = up[2];
        }
        rc = build_device_tree(dx, dy, dz, n, J, r, M, offset, domain4, t->h, &t->d_x, &t->d_y, &t->d_z, &t->d_orig,
                               err);
        for (double* p : up) if (p) (void)hipFree(p);
    } else {
        rc = build_host_tree(px, py, pz, n, J, r, M, offset, flags, domain4, t->h, err);
    }
    if (rc) { delete t; return fail(rc, err); }
    const HostTree& h = t->h;
    if (M - 1 + ((flags & MRA_FURTHER_APPROX) ? 1 : 0) > chain_lmax(h.P)) {
        delete t;
        return fail(MRA_EINVAL, "M - 1 = " + std::to_string(M - 1) + " exceeds " + std::to_string(chain_lmax(h.P)) +
                                    " levels above the finest");
    }
    t->WF = (M - 1) * h.P + 1;
    t->fa_cols = (flags & MRA_FURTHER_APPROX) ? h.P : 0;
    t->WFs = (t->fa_cols + t->WF + 15) & ~15;  // rows of whole 128-byte lines
    t->leaf_min = INT64_MAX;
    for (int64_t g = h.lvl_start[M - 1]; g < h.lvl_start[M]; ++g) {
        const int64_t nc = h.obs_hi[g] - h.obs_lo[g];
        t->leaf_min = std::min(t->leaf_min, nc);
        t->leaf_max = std::max(t->leaf_max, nc);
        int b = 0;
        while (b < 15 && (int64_t(1) << b) <= nc) ++b;  // 2^(b-1) <= nc < 2^b
        ++t->leaf_hist[b];
    }
    if (t->leaf_min == INT64_MAX) t->leaf_min = 0;
    t->opts.fold_max.assign(M, -1);
    t->opts.tile.assign(M, -1);
    if ((rc = make_plan(h, flags, false, nullptr, &t->opts, t->lik, err))) {
        delete t;
        return fail(rc, err);
    }
    std::vector<int64_t> lo(h.obs_lo), hi(h.obs_hi);
    if ((!on_gpu && ((rc = upload(&t->d_x, h.x)) || (rc = upload(&t->d_y, h.y)) || (rc = upload(&t->d_z, h.z)))) ||
        (rc = upload(&t->d_box, h.box)) || (rc = upload(&t->d_obs_lo, lo)) || (rc = upload(&t->d_obs_hi, hi))) {
        delete t;
        return fail(rc, "device allocation or copy failed while uploading the tree");
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
    info->n_gram_regions = t->lik.n_gram;
    info->n_dup = h.n_dup;
    for (int b = 0; b < 16; ++b) info->leaf_hist[b] = t->leaf_hist[b];
    return MRA_OK;
}

extern "C" int mra_tree_arrays(const mra_tree* t, double* x, double* y, double* z, int64_t* orig,
                               int64_t* leaf_off) {
    if (!t) return fail(MRA_EINVAL, "NULL tree");
    const HostTree& h = t->h;
    const size_t n = size_t(h.n_used);
    if (t->d_orig) {  // built on the GPU: the grouped observations live on the device
        if ((x && n && hipMemcpy(x, t->d_x, n * 8, hipMemcpyDeviceToHost) != hipSuccess) ||
            (y && n && hipMemcpy(y, t->d_y, n * 8, hipMemcpyDeviceToHost) != hipSuccess) ||
            (z && n && hipMemcpy(z, t->d_z, n * 8, hipMemcpyDeviceToHost) != hipSuccess) ||
            (orig && n && hipMemcpy(orig, t->d_orig, n * 8, hipMemcpyDeviceToHost) != hipSuccess))
            return fail(MRA_EDEVICE, "copy of the tree's observations failed");
    } else {
        if (x) std::memcpy(x, h.x.data(), n * 8);
        if (y) std::memcpy(y, h.y.data(), n * 8);
        if (z) std::memcpy(z, h.z.data(), n * 8);
        if (orig) std::memcpy(orig, h.orig.data(), n * 8);
    }
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
    if (family == MRA_MATERN && nu == 2.5) { *smooth = 2; return MRA_OK; }
    if (family == MRA_GAUSS) { *smooth = 3; return MRA_OK; }
    return fail(MRA_EINVAL, "family must be MRA_EXP, MRA_MATERN with nu 0.5, 1.5 or 2.5, or MRA_GAUSS");
}

static int region_level(const HostTree& h, int64_t g) {
    for (int m = 1; m <= h.M; ++m) if (g < h.lvl_start[m]) return m;
    return h.M;
}

// MRA_OK, or MRA_ENOTPD naming the first theta whose factorisation failed
// (status: per theta 0 or 1 + the global index of the failing region).
static int status_message(const HostTree& h, const int* status, int64_t B) {
    for (int64_t b = 0; b < B; ++b)
        if (status[b] < 0)
            return fail(MRA_EDEVICE, "theta " + std::to_string(b) +
                                         ": a finisher's bounded wait for the theta sharing its prior ran out");
    for (int64_t b = 0; b < B; ++b)
        if (status[b] != 0) {
            const int64_t g = status[b] - 1;
            const int lev = region_level(h, g);
            return fail(MRA_ENOTPD, "not positive definite: theta " + std::to_string(b) + ", level " +
                                        std::to_string(lev) + ", region " + std::to_string(g - h.lvl_start[lev - 1]));
        }
    return MRA_OK;
}

static bool theta_ok(const double* q, bool zero_nugget = false) {
    return q[0] > 0.0 && q[1] > 0.0 && (q[2] > 0.0 || (zero_nugget && q[2] == 0.0)) && std::isfinite(q[0]) &&
           std::isfinite(q[1]) && std::isfinite(q[2]);
}

// Kernel arguments common to every launch over a tree and plan.
static KArgs base_args(const mra_tree* t, const Plan& pl, int smooth) {
    const HostTree& h = t->h;
    KArgs a{};
    a.x = t->d_x; a.y = t->d_y; a.z = t->d_z; a.box = t->d_box;
    a.obs_lo = t->d_obs_lo; a.obs_hi = t->d_obs_hi;
    a.vst_off = pl.d_vst_off; a.gram_off = pl.d_gram_off; a.form = pl.d_form;
    for (int m = 0; m <= h.M && m <= MAXL; ++m) a.lvl[m] = h.lvl_start[m];
    a.J = h.J; a.M = h.M; a.nx = h.nx; a.ny = h.ny; a.rhat = h.rhat; a.P = h.P; a.WF = t->WF; a.WFs = t->WFs;
    a.offset = h.offset; a.smooth = smooth;
    a.vst_stride = pl.vst_size;
    a.F_stride = std::max<int64_t>(h.n_used, 1) * t->WFs;
    a.gram_stride = pl.gram_size;
    a.d_stride = h.nreg;
    a.n_used = double(h.n_used);
    a.zero_nugget = (t->flags & MRA_ALLOW_ZERO_NUGGET) ? 1 : 0;
    a.fa = t->fa_cols > 0 ? 1 : 0;
    a.rep = nullptr;
    a.leaf_phase = -1;
    a.order = a.need = nullptr;
    a.wait = a.queue = nullptr;
    a.S0 = nullptr;
    a.S0_off = pl.d_s0_off;
    a.S0_stride = pl.s0_size;
    return a;
}

// Prior (levels 1..M-1) and the observations' whitened rows for one chunk.
// nth: theta the prior is computed for (the flop count of the profiler).
static hipError_t enqueue_prior(const mra_tree* t, const Plan& pl, KArgs a, int nb, hipStream_t st, double nth = -1) {
    if (nth < 0) nth = nb;
    const int M = t->h.M;
    hipError_t e;
    const int Mk = a.fa ? M : M - 1;  // levels with knots
    for (int m = 1; m <= Mk; ++m) {
        a.level = m;
        a.tasks = pl.d_prior[m];
        a.ntasks = int64_t(pl.prior_tasks[m].size());
        if (a.ntasks == 0) continue;
        const int grid = int(std::min<int64_t>(a.ntasks * nb, 1 << 16));
        if (m > 1 && (e = timed(0, m, pl.fl_chain[m] * nth, st, [&] { return launch_chain(a, 0, grid, st); }))) return e;
        if ((e = timed(1, m, pl.fl_pfin[m] * nth, st, [&] { return launch_prior_finish(a, grid, st); }))) return e;
    }
    if (Mk >= 1 && !pl.chain_obs_tasks.empty()) {
        a.level = M - 1 + a.fa;
        a.tasks = pl.d_chain_obs;
        a.ntasks = int64_t(pl.chain_obs_tasks.size());
        const int grid = int(std::min<int64_t>(a.ntasks * nb, 1 << 16));
        if ((e = timed(0, M, pl.fl_chain_obs * nth, st, [&] { return launch_chain(a, 1, grid, st); }))) return e;
    }
    return hipSuccess;
}

// Finest-level factors of the observations for one chunk.
// nth: theta whose tasks run in this launch sequence (the flop count).
// leaf_phase 3: the one-wave finishers run phase 0 and then phase 1, the
// workgroup finisher runs every theta in one launch (see KArgs::wait).
static hipError_t enqueue_leaves(const mra_tree* t, const Plan& pl, KArgs a, int nb, int64_t nslot, hipStream_t st,
                                 double nth = -1, double nrep = 0) {
    if (nth < 0) nth = nb;
    const int M = t->h.M;
    hipError_t e;
    a.level = M;
    const int phase = a.leaf_phase;
    for (int q = 0; q < 3; ++q) {
        a.tasks = pl.d_small[q];
        a.ntasks = int64_t(pl.small_tasks[q].size());
        const double fq = phase == 2 ? pl.fl_small_s[q] : phase >= 0 ? pl.fl_small[q] - pl.fl_small_s[q]
                                                                     : pl.fl_small[q];
        for (int ph : phase == 3 ? std::initializer_list<int>{0, 1} : std::initializer_list<int>{phase}) {
            a.leaf_phase = ph;
            const double nq = phase != 3 ? nth : ph == 0 ? nb - nrep : nrep;
            if (a.ntasks > 0 && (e = timed(6, M, fq * nq, st, [&] {
                                     return launch_small(a, 16 << q, 0, int(std::min<int64_t>(a.ntasks * nb, 1 << 18)), st);
                                 })))
                return e;
        }
        a.leaf_phase = phase;
    }
    a.tasks = pl.d_leaf;
    a.ntasks = int64_t(pl.leaf_tasks.size());
    const double fl = a.leaf_phase == 2 ? pl.fl_leaf_s : a.leaf_phase >= 0 ? pl.fl_leaf - pl.fl_leaf_s : pl.fl_leaf;
    if (phase == 3 && a.ntasks > 0 && (e = launch_fill_int(a.wait, a.ntasks * nb, 0, st))) return e;
    if (a.ntasks > 0 && (e = timed(2, M, fl * nth, st, [&] {
                             return launch_leaf(a, int(std::min<int64_t>(a.ntasks * nb, nslot)), st);
                         })))
        return e;
    return hipSuccess;
}

// Fold of level m for one chunk.
static hipError_t enqueue_fold(const mra_tree* t, const Plan& pl, KArgs a, int m, int nb, int64_t nslot,
                               hipStream_t st) {
    (void)t;
    hipError_t e;
    a.level = m;
    for (int q = 0; q < 3; ++q) {
        a.tasks = pl.d_fsmall[q][m];
        a.ntasks = int64_t(pl.fsmall_tasks[q][m].size());
        if (a.ntasks > 0 && (e = timed(7, m, pl.fl_fsmall[q][m] * nb, st, [&] {
                                 return launch_small(a, 16 << q, 1, int(std::min<int64_t>(a.ntasks * nb, 1 << 18)), st);
                             })))
            return e;
    }
    a.tasks = pl.d_factor[m];
    a.ntasks = int64_t(pl.factor_tasks[m].size());
    if (a.ntasks > 0 && (e = timed(3, m, pl.fl_factor[m] * nb, st, [&] {
                             return launch_fold_factor(a, int(std::min<int64_t>(a.ntasks * nb, nslot)), st);
                         })))
        return e;
    a.tasks = pl.d_gramt[m];
    a.ntasks = int64_t(pl.gram_tasks[m].size());
    if (a.ntasks > 0) {
        if ((e = timed(4, m, pl.fl_gram[m] * nb, st, [&] {
                 return launch_gram_panel(a, int(std::min<int64_t>(a.ntasks * nb, 1 << 16)), st);
             })))
            return e;
        if (m > 1 && (e = timed(pl.gtile_super[m] ? 11 : 10, m, pl.fl_gtile[m] * nb, st, [&] {
                          return pl.gtile_super[m] ? launch_gram_tile2(a, st) : launch_gram_tile(a, st);
                      })))
            return e;
    }
    return hipSuccess;
}

#define HIPCHK(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) {                                                                           \
            rc = fail(MRA_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));                      \
            goto done;                                                                                    \
        }                                                                                                 \
    } while (0)

// Device workspace of a tree, kept between calls (allocation of the large
// buffers is not repeated per evaluation).  Calls on one tree are serialised:
// a call on a different stream first waits for the previous call's work.
struct Workspace {
    double *vst = nullptr, *F = nullptr, *gram = nullptr, *dval = nullptr, *scratch = nullptr;
    double *th = nullptr, *out = nullptr, *ld = nullptr, *q = nullptr;
    int* status = nullptr;
    int* rep = nullptr;  // per theta of a chunk: its representative, the finisher's order, group sizes
    int* wait = nullptr;   // per leaf task and theta of a chunk: the group's count (merged leaf launch)
    int* queue = nullptr;  // the finishers' work-queue counters
    double* S0 = nullptr;  // per theta of a chunk: C - V V^T of every leaf (shared prior)
    int64_t Bc = 0, nslot = 0, scratch_per = 0, cap_B = 0;
    bool mem_limited = false;  // Bc was capped by device memory, not by the request
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    int64_t last_B = 0;          // theta of the most recent evaluation (its status in `status`)
    const double* last_th = nullptr;  // its device theta
    // captured graphs of whole evaluations, keyed by (theta, out, logdet, quad, B, smooth, stream)
    std::map<std::tuple<const void*, void*, void*, void*, int64_t, int, void*>, hipGraphExec_t> graphs;
    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    void release() {
        if (done) { (void)hipEventSynchronize(done); (void)hipEventDestroy(done); done = nullptr; }
        drop_graphs();
        for (void* p : {static_cast<void*>(vst), static_cast<void*>(F), static_cast<void*>(gram),
                        static_cast<void*>(dval), static_cast<void*>(scratch), static_cast<void*>(th),
                        static_cast<void*>(out), static_cast<void*>(ld), static_cast<void*>(q),
                        static_cast<void*>(status), static_cast<void*>(rep), static_cast<void*>(S0),
                        static_cast<void*>(wait), static_cast<void*>(queue)})
            if (p) (void)hipFree(p);
        vst = F = gram = dval = scratch = th = out = ld = q = S0 = nullptr;
        status = rep = wait = queue = nullptr;
        Bc = nslot = cap_B = 0;
        used = false;
    }
};

static std::mutex g_ws_mu;

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
    void* ps[] = {d_x, d_y, d_z, d_box, d_obs_lo, d_obs_hi, d_orig};
    for (void* p : ps)
        if (p) (void)hipFree(p);
}

static int ensure_workspace(const mra_tree* t, Workspace& w, int64_t B, hipStream_t st) {
    const HostTree& h = t->h;
    const Plan& pl = t->lik;
    const int64_t F_stride = std::max<int64_t>(h.n_used, 1) * t->WFs;
    const int64_t per_theta = pl.vst_size + F_stride + pl.gram_size + h.nreg + pl.s0_size;
    const int64_t scratch_per = (std::max<int64_t>({pl.scratch_leaf, pl.scratch_fold, 1}) + 31) & ~int64_t(31);
    // reuse when the buffers hold enough theta per chunk (or could not hold more)
    if (w.Bc > 0 && w.cap_B >= B && (w.Bc >= B || w.mem_limited)) return MRA_OK;
    if (w.Bc > 0) w.release();
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(MRA_EDEVICE, "hipMemGetInfo failed");
    const double budget = 0.6 * double(free_b) / 8.0;  // doubles
    const int64_t nslot = std::min<int64_t>(2048, std::max<int64_t>(1, int64_t(0.2 * budget / double(scratch_per))));
    const double left = budget - double(nslot) * double(scratch_per);
    int64_t Bc = std::min<int64_t>(std::max<int64_t>(B, 1), int64_t(left / double(per_theta)));
    if (Bc < 1) return fail(MRA_ENOMEM, "not enough device memory for one theta");
    // whole groups of theta that share a prior per chunk (when more than one fits)
    if (Bc < B && Bc >= t->chunk_multiple) Bc -= Bc % t->chunk_multiple;
    const int64_t capB = std::max<int64_t>(B, 64);
    auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 8)) == hipSuccess; };
    if (!al(reinterpret_cast<void**>(&w.vst), size_t(Bc) * pl.vst_size * 8) ||
        !al(reinterpret_cast<void**>(&w.F), size_t(Bc) * F_stride * 8) ||
        !al(reinterpret_cast<void**>(&w.gram), size_t(Bc) * pl.gram_size * 8) ||
        !al(reinterpret_cast<void**>(&w.dval), size_t(Bc) * h.nreg * 8) ||
        !al(reinterpret_cast<void**>(&w.scratch), size_t(nslot) * scratch_per * 8) ||
        !al(reinterpret_cast<void**>(&w.status), size_t(capB) * sizeof(int)) ||
        !al(reinterpret_cast<void**>(&w.rep), (size_t(capB) * 3 + 1) * sizeof(int)) ||
        !al(reinterpret_cast<void**>(&w.wait), size_t(Bc) * pl.leaf_tasks.size() * sizeof(int)) ||
        !al(reinterpret_cast<void**>(&w.queue), 2 * sizeof(int)) ||
        !al(reinterpret_cast<void**>(&w.S0), size_t(Bc) * pl.s0_size * 8) ||
        !al(reinterpret_cast<void**>(&w.th), size_t(capB) * 3 * 8) ||
        !al(reinterpret_cast<void**>(&w.out), size_t(capB) * 8) ||
        !al(reinterpret_cast<void**>(&w.ld), size_t(capB) * 8) ||
        !al(reinterpret_cast<void**>(&w.q), size_t(capB) * 8)) {
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

// Every launch of one evaluation of B parameter vectors, in chunks of Bc
// theta (the per-theta buffers of a.vst, a.F, a.gram, a.dval hold Bc theta;
// nslot workgroup slots of a.scratch).  With rep_buf (Bc ints on the device),
// theta of a chunk that share alpha and range share the prior: it is computed
// for the first of them (the representative), the others' finest-level
// finishers read its rows before the representative's own finisher
// overwrites them.  Which theta share is found on the device, so that a
// captured graph stays valid for new values in the same buffer.
static hipError_t enqueue_loglik(const mra_tree* t, int64_t Bc, int64_t nslot, KArgs a, const double* d_th,
                                 double* d_out, double* d_ld, double* d_q, int* status, int64_t B, hipStream_t st,
                                 double* d_lev = nullptr, int* rep_buf = nullptr, double* s0_buf = nullptr) {
    const HostTree& h = t->h;
    const Plan& pl = t->lik;
    hipError_t e;
    bool prof;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof = g_prof_on;
    }
    if ((e = launch_fill_int(status, B, 0, st))) return e;
    if (a.queue && (e = launch_fill_int(a.queue, 2, 0, st))) return e;
    for (int64_t b0 = 0; b0 < B; b0 += Bc) {
        const int nb = int(std::min<int64_t>(Bc, B - b0));
        a.theta = d_th + 3 * b0;
        a.ntheta = nb;
        a.status = status + b0;
        a.out = d_out + b0;
        a.out_ld = d_ld ? d_ld + b0 : nullptr;
        a.out_q = d_q ? d_q + b0 : nullptr;
        a.out_lev = d_lev ? d_lev + b0 * h.M : nullptr;
        const bool share = rep_buf && s0_buf && nb > 1 && h.M > 1;
        double nrep = nb;  // representatives (the profiler's flop count; eager launches only)
        if (share && prof) {
            std::vector<double> th(size_t(3) * nb);
            if ((e = hipMemcpyAsync(th.data(), a.theta, th.size() * 8, hipMemcpyDeviceToHost, st))) return e;
            if ((e = hipStreamSynchronize(st))) return e;
            nrep = 0;
            for (int i = 0; i < nb; ++i) {
                bool first = true;
                for (int j = 0; j < i && first; ++j)
                    first = !(th[3 * j] == th[3 * i] && th[3 * j + 1] == th[3 * i + 1]);
                nrep += first ? 1 : 0;
            }
        }
        a.rep = nullptr;
        a.leaf_phase = -1;
        if (share) {
            if ((e = launch_rep(a.theta, nb, rep_buf, st))) return e;
            a.rep = rep_buf;
        }
        if ((e = launch_fill(a.dval, int64_t(nb) * a.d_stride, 0.0, st))) return e;
        if ((e = enqueue_prior(t, pl, a, nb, st, nrep))) return e;
        if (share) {
            if ((e = launch_rep_status(a.rep, nb, a.status, st))) return e;
            a.S0 = s0_buf;
            a.leaf_phase = 2;  // C - V V^T of every leaf, once per representative
            if ((e = enqueue_leaves(t, pl, a, nb, nslot, st, nrep))) return e;
            // the theta that share a prior from their representative's rows,
            // then the representatives in place (the workgroup finisher: in
            // one launch, which needs the work queue)
            if (a.queue && a.wait) {
                a.leaf_phase = 3;
                a.order = rep_buf + nb;
                a.need = rep_buf + 2 * nb;
                if ((e = enqueue_leaves(t, pl, a, nb, nslot, st, nb, nrep))) return e;
            } else {
                a.leaf_phase = 0;
                if ((e = enqueue_leaves(t, pl, a, nb, nslot, st, nb - nrep))) return e;
                a.leaf_phase = 1;
                if ((e = enqueue_leaves(t, pl, a, nb, nslot, st, nrep))) return e;
            }
            a.rep = a.order = a.need = nullptr;
            a.S0 = nullptr;
            a.leaf_phase = -1;
        } else if ((e = enqueue_leaves(t, pl, a, nb, nslot, st))) {
            return e;
        }
        for (int m = h.M - 1; m >= 1; --m)
            if ((e = enqueue_fold(t, pl, a, m, nb, nslot, st))) return e;
        if ((e = timed(5, 0, 0.0, st, [&] { return launch_final(a, h.nreg, pl.root_gram, st); }))) return e;
    }
    return hipSuccess;
}

// Sharing of the prior between theta with the same alpha and range is on
// unless MRA_SHARE_PRIOR=0.
static bool share_enabled() {
    const char* e = std::getenv("MRA_SHARE_PRIOR");
    return !(e && *e == '0');
}

// Repeated evaluations with device pointers on a non-null stream replay a
// captured graph of the whole launch sequence (MRA_GRAPHS=0 disables this).
static bool graphs_enabled() {
    const char* e = std::getenv("MRA_GRAPHS");
    return !(e && *e == '0');
}

static int loglik_impl(const mra_tree* t, int family, double nu, const double* theta, int64_t B, double* loglik,
                       double* logdet, double* quad, void* stream, double* levels = nullptr) {
    if (!t || !theta || !loglik || B < 1) return fail(MRA_EINVAL, "NULL argument or B < 1");
    int smooth = 0;
    int rc = smooth_of(family, nu, &smooth);
    if (rc) return rc;
    const HostTree& h = t->h;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const bool dev = is_device_ptr(theta);
    if (dev != is_device_ptr(loglik) || (logdet && dev != is_device_ptr(logdet)) || (quad && dev != is_device_ptr(quad)) ||
        (levels && dev != is_device_ptr(levels)))
        return fail(MRA_EINVAL, "theta and the outputs must be in the same memory space");
    const bool zn = (t->flags & MRA_ALLOW_ZERO_NUGGET) != 0;
    if (!dev)
        for (int64_t b = 0; b < B; ++b)
            if (!theta_ok(theta + 3 * b, zn))
                return fail(MRA_EINVAL, "theta " + std::to_string(b) + ": alpha, beta, tau must be finite and > 0" +
                                            (zn ? " (tau >= 0)" : ""));

    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace& w = workspace_of(t);
    rc = ensure_workspace(t, w, B, st);
    if (rc) return rc;
    if (w.used && w.last != st) (void)hipStreamWaitEvent(st, w.done, 0);
    double* d_th = dev ? const_cast<double*>(theta) : w.th;
    double* d_out = dev ? loglik : w.out;
    double* d_ld = logdet ? (dev ? logdet : w.ld) : nullptr;
    double* d_q = quad ? (dev ? quad : w.q) : nullptr;
    double* d_lev = nullptr;
    if (levels && !dev) {
        if (hipMallocAsync(reinterpret_cast<void**>(&d_lev), size_t(B) * h.M * 8, st) != hipSuccess)
            return fail(MRA_ENOMEM, "device allocation of the per-level sums failed");
    } else if (levels) {
        d_lev = levels;
    }
    std::vector<int> hstatus;
    KArgs a = base_args(t, t->lik, smooth);
    a.vst = w.vst; a.F = w.F + t->fa_cols; a.gram = w.gram; a.dval = w.dval;
    a.scratch = w.scratch; a.scratch_stride = w.scratch_per;
    a.queue = w.queue; a.wait = w.wait;
    bool profiling;
    {
        std::lock_guard<std::mutex> pk(g_prof_mu);
        profiling = g_prof_on;
    }
    const bool share = share_enabled();
    int* rep_buf = share ? w.rep : nullptr;
    if (!dev) HIPCHK(hipMemcpyAsync(d_th, theta, 3 * B * 8, hipMemcpyHostToDevice, st));
    if (dev && st != nullptr && !profiling && graphs_enabled() && !levels) {
        // a repeated evaluation on the same buffers replays one captured graph
        const auto key = std::make_tuple(static_cast<const void*>(theta), static_cast<void*>(loglik),
                                         static_cast<void*>(logdet), static_cast<void*>(quad), B,
                                         smooth + (share ? 16 : 0), static_cast<void*>(st));
        auto it = w.graphs.find(key);
        if (it == w.graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const hipError_t ce =
                enqueue_loglik(t, w.Bc, w.nslot, a, d_th, d_out, d_ld, d_q, w.status, B, st, nullptr, rep_buf, w.S0);
            const hipError_t ee = hipStreamEndCapture(st, &g);
            HIPCHK(ce);
            HIPCHK(ee);
            const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCHK(ie);
            it = w.graphs.emplace(key, ge).first;
        }
        HIPCHK(hipGraphLaunch(it->second, st));
    } else {
        HIPCHK(enqueue_loglik(t, w.Bc, w.nslot, a, d_th, d_out, d_ld, d_q, w.status, B, st, d_lev, rep_buf, w.S0));
    }
    (void)hipEventRecord(w.done, st);
    w.last = st;
    w.used = true;
    w.last_B = B;
    w.last_th = d_th;
    if (!dev) {
        HIPCHK(hipMemcpyAsync(loglik, d_out, B * 8, hipMemcpyDeviceToHost, st));
        if (logdet) HIPCHK(hipMemcpyAsync(logdet, d_ld, B * 8, hipMemcpyDeviceToHost, st));
        if (quad) HIPCHK(hipMemcpyAsync(quad, d_q, B * 8, hipMemcpyDeviceToHost, st));
        if (levels) HIPCHK(hipMemcpyAsync(levels, d_lev, size_t(B) * h.M * 8, hipMemcpyDeviceToHost, st));
        hstatus.resize(B);
        HIPCHK(hipMemcpyAsync(hstatus.data(), w.status, B * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        rc = status_message(h, hstatus.data(), B);
    }
done:
    if (d_lev && d_lev != levels) (void)hipFreeAsync(d_lev, st);
    return rc;
}

extern "C" int mra_loglik_status(const mra_tree* t) {
    if (!t) return fail(MRA_EINVAL, "NULL tree");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (!t->ws) return fail(MRA_EINVAL, "no evaluation on this tree");
    Workspace& w = *static_cast<Workspace*>(t->ws);
    if (!w.used || w.last_B < 1) return fail(MRA_EINVAL, "no evaluation on this tree");
    if (hipEventSynchronize(w.done) != hipSuccess) return fail(MRA_EDEVICE, "waiting for the evaluation failed");
    std::vector<int> hs(w.last_B);
    std::vector<double> th(3 * w.last_B);
    if (hipMemcpy(hs.data(), w.status, w.last_B * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(th.data(), w.last_th, 3 * w.last_B * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MRA_EDEVICE, "copy of the evaluation status failed");
    const bool zn = (t->flags & MRA_ALLOW_ZERO_NUGGET) != 0;
    for (int64_t b = 0; b < w.last_B; ++b)
        if (!theta_ok(&th[3 * b], zn))
            return fail(MRA_EINVAL, "theta " + std::to_string(b) + ": alpha, beta, tau must be finite and > 0");
    return status_message(t->h, hs.data(), w.last_B);
}

extern "C" int mra_loglik(const mra_tree* t, int family, double nu, const double* theta, int64_t B,
                          double* loglik, void* stream) {
    return loglik_impl(t, family, nu, theta, B, loglik, nullptr, nullptr, stream);
}

extern "C" int mra_loglik_terms(const mra_tree* t, int family, double nu, const double* theta, int64_t B,
                                double* loglik, double* logdet, double* quad, void* stream) {
    return loglik_impl(t, family, nu, theta, B, loglik, logdet, quad, stream);
}

extern "C" int mra_loglik_levels(const mra_tree* t, int family, double nu, const double* theta, int64_t B,
                                 double* loglik, double* level_logdet, void* stream) {
    if (!level_logdet) return fail(MRA_EINVAL, "level_logdet is NULL");
    return loglik_impl(t, family, nu, theta, B, loglik, nullptr, nullptr, stream, level_logdet);
}

// ------------------------------------------- evaluation without allocation

// Device memory of mra_loglik_noalloc: one array per GPU, kept until the
// process ends.  In host code `scratch` is only a symbol; its device address
// is looked up once per device (hipGetSymbolAddress) and that address is what
// the kernels receive.
constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) double scratch[NOALLOC_BYTES / sizeof(double)];

static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[64] = {nullptr};

static int noalloc_base(int dev, double** out) {
    if (dev < 0 || dev >= 64) return fail(MRA_EDEVICE, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MRA_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                         hipGetErrorString(e));
        g_noalloc_ptr[dev] = p;
    }
    *out = static_cast<double*>(g_noalloc_ptr[dev]);
    return MRA_OK;
}

extern "C" int mra_loglik_noalloc(const mra_tree* t, int family, double nu, const double* theta, int64_t B,
                                  double* loglik, void* stream) {
    if (!t || !theta || !loglik || B < 1) return fail(MRA_EINVAL, "NULL argument or B < 1");
    int smooth = 0;
    int rc = smooth_of(family, nu, &smooth);
    if (rc) return rc;
    if (!is_device_ptr(theta) || !is_device_ptr(loglik))
        return fail(MRA_EINVAL, "mra_loglik_noalloc takes device pointers for theta and loglik");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MRA_EDEVICE, "hipGetDevice failed");
    if (dev != t->device) return fail(MRA_EINVAL, "the current device is not the tree's device");
    double* base = nullptr;
    if ((rc = noalloc_base(dev, &base))) return rc;
    const HostTree& h = t->h;
    const Plan& pl = t->lik;
    // layout (doubles, each part 256-byte aligned): status (B ints) and the
    // finishers' queue counters, then Bc theta of V stores, F rows, Gram
    // blocks and log-determinants, then nslot workgroup slots
    auto al32 = [](int64_t v) { return (v + 31) & ~int64_t(31); };
    const int64_t cap = int64_t(NOALLOC_BYTES / sizeof(double));
    const int64_t st_sz = al32((B * int64_t(sizeof(int)) + 7) / 8) + 32;
    const int64_t F_stride = std::max<int64_t>(h.n_used, 1) * t->WFs;
    const int64_t per_theta = al32(pl.vst_size) + al32(F_stride) + al32(pl.gram_size) + al32(h.nreg);
    const int64_t slot = al32(std::max<int64_t>({pl.scratch_leaf, pl.scratch_fold, 1}));
    int64_t nslot = 256;
    while (nslot > 1 && st_sz + per_theta + nslot * slot > cap) nslot /= 2;
    if (st_sz + per_theta + nslot * slot > cap)
        return fail(MRA_ENOMEM, "mra_loglik_noalloc: one theta of this tree needs " +
                                    std::to_string((st_sz + per_theta + slot) * 8) + " bytes of scratch, the limit is " +
                                    std::to_string(NOALLOC_BYTES) + " bytes");
    const int64_t Bc = std::min<int64_t>(B, (cap - st_sz - nslot * slot) / per_theta);
    KArgs a = base_args(t, pl, smooth);
    int* status = reinterpret_cast<int*>(base);
    a.queue = reinterpret_cast<int*>(base + st_sz - 32);  // zeroed at the start of the launch sequence
    double* p = base + st_sz;
    a.vst = p; p += Bc * al32(pl.vst_size);
    a.F = p + t->fa_cols; p += Bc * al32(F_stride);
    a.gram = p; p += Bc * al32(pl.gram_size);
    a.dval = p; p += Bc * al32(h.nreg);
    a.scratch = p;
    a.scratch_stride = slot;
    a.vst_stride = al32(pl.vst_size);
    a.F_stride = al32(F_stride);
    a.gram_stride = al32(pl.gram_size);
    a.d_stride = al32(h.nreg);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    t_untimed = true;
    const hipError_t e = enqueue_loglik(t, Bc, nslot, a, theta, loglik, nullptr, nullptr, status, B, st);
    t_untimed = false;
    if (e != hipSuccess) return fail(MRA_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return MRA_OK;
}

// ------------------------------------------------------------- autotuning

// Rebuild the likelihood plan of a tree from its options; the evaluation
// workspace (sized by the plan) and its captured graphs are dropped.
static int replan(mra_tree* t) {
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        if (t->ws) static_cast<Workspace*>(t->ws)->release();
    }
    t->lik.~Plan();
    new (&t->lik) Plan();
    std::string err;
    const int rc = make_plan(t->h, t->flags, false, nullptr, &t->opts, t->lik, err);
    return rc ? fail(rc, err) : MRA_OK;
}

extern "C" int mra_set_tile_shapes(mra_tree* t, const int32_t* tile) {
    if (!t) return fail(MRA_EINVAL, "NULL tree");
    const int M = t->h.M;
    for (int m = 1; m < M; ++m) {
        const int32_t v = tile ? tile[m - 1] : -1;
        if (v < -1 || v > 1) return fail(MRA_EINVAL, "tile shapes must be -1, 0 or 1");
        t->opts.tile[m] = int8_t(v);
    }
    return replan(t);
}

extern "C" int mra_set_chunk_multiple(mra_tree* t, int64_t multiple) {
    if (!t) return fail(MRA_EINVAL, "NULL tree");
    if (multiple < 1) return fail(MRA_EINVAL, "the chunk multiple must be at least 1");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (t->ws) static_cast<Workspace*>(t->ws)->release();
    t->chunk_multiple = multiple;
    return MRA_OK;
}

extern "C" int mra_set_plan(mra_tree* t, const int64_t* fold_max, int small_max) {
    if (!t) return fail(MRA_EINVAL, "NULL tree");
    if (small_max != 16 && small_max != 32 && small_max != 64) return fail(MRA_EINVAL, "small_max must be 16, 32 or 64");
    const int M = t->h.M;
    for (int m = 1; m < M; ++m) {
        const int64_t v = fold_max ? fold_max[m - 1] : -1;
        if (v > (int64_t(1) << 14)) return fail(MRA_EINVAL, "fold_max above 16384 observations");
        t->opts.fold_max[m] = v < 0 ? -1 : v;
    }
    t->opts.small_max = small_max;
    return replan(t);
}

// Form of every level-m region under a candidate threshold, given the forms
// of the level below in the installed plan (to skip candidates that change
// nothing); the same rule as make_plan.
static std::vector<int8_t> level_forms(const HostTree& h, const std::vector<int8_t>& form, int m, int64_t thr) {
    std::vector<int8_t> f;
    for (int64_t g = h.lvl_start[m - 1]; g < h.lvl_start[m]; ++g) {
        const int64_t np = h.obs_hi[g] - h.obs_lo[g];
        bool fac = np <= thr;
        if (fac && m + 1 < h.M)
            for (int j = 0; j < h.J; ++j) {
                const int64_t gc = h.lvl_start[m] + (g - h.lvl_start[m - 1]) * h.J + j;
                if (h.obs_hi[gc] > h.obs_lo[gc] && form[gc] != FOLD_FACTOR) fac = false;
            }
        f.push_back(np == 0 ? int8_t(2) : (fac ? int8_t(FOLD_FACTOR) : int8_t(FOLD_GRAM)));
    }
    return f;
}

extern "C" int mra_autotune(mra_tree* t, int family, double nu, const double* theta, int64_t B,
                            mra_tune_result* out) {
    if (!t || !theta || !out || B < 1) return fail(MRA_EINVAL, "NULL argument or B < 1");
    if (is_device_ptr(theta)) return fail(MRA_EINVAL, "theta must be host memory");
    if (t->flags & (MRA_FOLD_GRAM | MRA_FOLD_FACTOR))
        return fail(MRA_EINVAL, "the tree was built with a fixed fold form (MRA_FOLD_GRAM or MRA_FOLD_FACTOR)");
    const HostTree& h = t->h;
    const int M = h.M;
    std::vector<double> ll(B);
    int trials = 0;
    // one evaluation of the sample, best of two (the first call after a
    // plan change also allocates the workspace and is not timed)
    auto time_plan = [&](double* ms) -> int {
        int rc = loglik_impl(t, family, nu, theta, B, ll.data(), nullptr, nullptr, nullptr);
        if (rc) return rc;
        double best = 1e300;
        for (int k = 0; k < 2; ++k) {
            const auto t0 = std::chrono::steady_clock::now();
            rc = loglik_impl(t, family, nu, theta, B, ll.data(), nullptr, nullptr, nullptr);
            if (rc) return rc;
            best = std::min(best, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        ++trials;
        *ms = best;
        return MRA_OK;
    };
    int rc;
    double ms_before = 0.0;
    if ((rc = time_plan(&ms_before))) return rc;
    double ms_best = ms_before;
    const int64_t cands[] = {0, 64, 128, 192, 256, 320, 384, 512, 768};
    // levels bottom-up: the finest folds hold most of the work
    for (int m = M - 1; m >= 1; --m) {
        const int64_t keep = t->opts.fold_max[m];
        const int64_t cur_thr = keep >= 0 ? keep : std::min<int64_t>(int64_t(m - 1) * h.P + 1, factor_fold_max());
        std::vector<std::vector<int8_t>> seen{level_forms(h, t->lik.form, m, cur_thr)};
        int64_t best_v = keep;
        for (int64_t c : cands) {
            auto f = level_forms(h, t->lik.form, m, c);
            if (std::find(seen.begin(), seen.end(), f) != seen.end()) continue;
            seen.push_back(f);
            t->opts.fold_max[m] = c;
            if ((rc = replan(t))) return rc;
            double ms = 0.0;
            if ((rc = time_plan(&ms))) return rc;
            if (ms < 0.98 * ms_best) { ms_best = ms; best_v = c; }
        }
        t->opts.fold_max[m] = best_v;
        if ((rc = replan(t))) return rc;
    }
    // the Schur blocks' tile shape per level with knot-space folds
    for (int m = M - 1; m >= 2; --m) {
        if (t->lik.gram_tasks[m].empty()) continue;
        const int8_t cur = t->lik.gtile_super[m];
        const int8_t keep = t->opts.tile[m];
        t->opts.tile[m] = cur ? 0 : 1;
        if ((rc = replan(t))) return rc;
        double ms = 0.0;
        if ((rc = time_plan(&ms))) return rc;
        if (ms < 0.98 * ms_best) ms_best = ms;
        else t->opts.tile[m] = keep;
    }
    if ((rc = replan(t))) return rc;
    for (int sm : {32, 16}) {
        const int keep = t->opts.small_max;
        t->opts.small_max = sm;
        if ((rc = replan(t))) return rc;
        double ms = 0.0;
        if ((rc = time_plan(&ms))) return rc;
        if (ms < 0.98 * ms_best) ms_best = ms;
        else t->opts.small_max = keep;
    }
    if ((rc = replan(t))) return rc;
    std::memset(out, 0, sizeof(*out));
    out->levels = M;
    for (int m = 1; m < M && m <= 16; ++m) {
        const int64_t v = t->opts.fold_max[m];
        out->fold_max[m - 1] = v >= 0 ? v : std::min<int64_t>(int64_t(m - 1) * h.P + 1, factor_fold_max());
    }
    out->small_max = t->opts.small_max;
    for (int m = 1; m < M && m <= 16; ++m) out->tile[m - 1] = t->lik.gtile_super[m];
    out->ms_before = ms_before;
    out->ms_after = ms_best;
    out->trials = trials;
    return MRA_OK;
}

// ---------------------------------------------------------------- kriging

extern "C" int mra_predict(const mra_tree* t, int family, double nu, const double* theta, const double* px,
                           const double* py, int64_t np, double* mean, double* var, void* stream) {
    if (!t || !theta || (np > 0 && (!px || !py || !mean || !var)) || np < 0)
        return fail(MRA_EINVAL, "NULL argument or np < 0");
    int smooth = 0;
    int rc = smooth_of(family, nu, &smooth);
    if (rc) return rc;
    if (t->fa_cols) return fail(MRA_EINVAL, "kriging is not provided for a tree built with MRA_FURTHER_APPROX");
    if (np == 0) return MRA_OK;
    const HostTree& h = t->h;
    const int M = h.M;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const bool dev = is_device_ptr(px);
    if (dev != is_device_ptr(py) || dev != is_device_ptr(mean) || dev != is_device_ptr(var) ||
        dev != is_device_ptr(theta))
        return fail(MRA_EINVAL, "theta, px, py, mean and var must all be host or all device pointers");
    double th[3];
    std::vector<double> hx(np), hy(np);
    if (dev) {
        if (hipMemcpy(th, theta, 24, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(hx.data(), px, np * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(hy.data(), py, np * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(MRA_EDEVICE, "copy of device inputs failed");
    } else {
        std::memcpy(th, theta, 24);
        std::memcpy(hx.data(), px, np * 8);
        std::memcpy(hy.data(), py, np * 8);
    }
    if (!theta_ok(th)) return fail(MRA_EINVAL, "alpha, beta, tau must be finite and > 0");
    for (int64_t i = 0; i < np; ++i)
        if (!std::isfinite(hx[i]) || !std::isfinite(hy[i])) return fail(MRA_EINVAL, "non-finite prediction location");
    std::string err;
    std::vector<int64_t> leaf;
    if ((rc = locate_leaves(h, hx.data(), hy.data(), np, leaf, err))) return fail(rc, err);
    // group the points by leaf (stable), ranges per region, counts per region
    const int64_t l0 = h.lvl_start[M - 1];
    std::vector<int64_t> cnt(h.nleaf + 1, 0);
    for (int64_t i = 0; i < np; ++i) ++cnt[leaf[i] - l0 + 1];
    for (int64_t k = 0; k < h.nleaf; ++k) cnt[k + 1] += cnt[k];
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1), perm(np), sleaf(np);
    std::vector<double> sx(np), sy(np);
    for (int64_t i = 0; i < np; ++i) {
        const int64_t d = fill[leaf[i] - l0]++;
        sx[d] = hx[i]; sy[d] = hy[i]; perm[d] = i; sleaf[d] = leaf[i];
    }
    std::vector<int64_t> plo(h.nreg), phi(h.nreg), pcount(h.nreg);
    for (int m = 0; m < M; ++m) {
        const int64_t span = ipow_h(h.J, M - 1 - m);
        for (int64_t k = 0; k < ipow_h(h.J, m); ++k) {
            const int64_t g = h.lvl_start[m] + k;
            plo[g] = cnt[k * span];
            phi[g] = cnt[(k + 1) * span];
            pcount[g] = phi[g] - plo[g];
        }
    }
    Plan pl;
    if ((rc = make_plan(h, t->flags, true, &pcount, &t->opts, pl, err))) return fail(rc, err);
    std::vector<int> pred_leaf_tasks, pred_chain_tasks;
    for (int64_t g = h.lvl_start[M - 1]; g < h.lvl_start[M]; ++g)
        if (pcount[g] > 0) pred_leaf_tasks.push_back(int(g));
    if (M > 1)
        for (int64_t g = h.lvl_start[M - 2]; g < h.lvl_start[M - 1]; ++g)
            if (pcount[g] > 0) pred_chain_tasks.push_back(int(g));
    int64_t kmax = 0, nmax = 0;
    for (int g : pred_leaf_tasks) {
        kmax = std::max(kmax, pcount[g]);
        nmax = std::max(nmax, h.obs_hi[g] - h.obs_lo[g]);
    }
    // device buffers (one theta)
    const int64_t F_stride = std::max<int64_t>(h.n_used, 1) * t->WFs;
    const int64_t scratch_per =
        (std::max<int64_t>({pl.scratch_leaf, pl.scratch_fold, nmax * nmax + nmax * (t->WFs + kmax), 1}) + 31) & ~int64_t(31);
    const int64_t nslot = 256;
    double *d_th = nullptr, *vst = nullptr, *F = nullptr, *gram = nullptr, *dval = nullptr, *scratch = nullptr,
           *PV = nullptr, *PS = nullptr, *PVAR = nullptr, *d_px = nullptr, *d_py = nullptr, *d_mean = nullptr,
           *d_var = nullptr, *out1 = nullptr;
    int* status = nullptr;
    int64_t *d_plo = nullptr, *d_phi = nullptr, *d_sleaf = nullptr, *d_perm = nullptr;
    int *d_pleaf = nullptr, *d_pchain = nullptr;
    int hstatus = 0;
    KArgs a = base_args(t, pl, smooth);
    std::vector<double> thv(th, th + 3);
    auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 8)) == hipSuccess; };
    if (!al(reinterpret_cast<void**>(&vst), pl.vst_size * 8) || !al(reinterpret_cast<void**>(&F), F_stride * 8) ||
        !al(reinterpret_cast<void**>(&gram), pl.gram_size * 8) || !al(reinterpret_cast<void**>(&dval), h.nreg * 8) ||
        !al(reinterpret_cast<void**>(&scratch), nslot * scratch_per * 8) ||
        !al(reinterpret_cast<void**>(&PV), np * t->WFs * 8) || !al(reinterpret_cast<void**>(&PS), np * t->WFs * 8) ||
        !al(reinterpret_cast<void**>(&PVAR), np * 8) || !al(reinterpret_cast<void**>(&status), sizeof(int)) ||
        !al(reinterpret_cast<void**>(&out1), 8) || upload(&d_th, thv) || upload(&d_px, sx) || upload(&d_py, sy) ||
        upload(&d_plo, plo) || upload(&d_phi, phi) || upload(&d_sleaf, sleaf) || upload(&d_perm, perm) ||
        upload(&d_pleaf, pred_leaf_tasks) || upload(&d_pchain, pred_chain_tasks) ||
        (!dev && (!al(reinterpret_cast<void**>(&d_mean), np * 8) || !al(reinterpret_cast<void**>(&d_var), np * 8)))) {
        (void)hipGetLastError();
        rc = fail(MRA_ENOMEM, "device allocation for prediction failed");
        goto done;
    }
    a.vst = vst; a.F = F; a.gram = gram; a.dval = dval; a.scratch = scratch; a.scratch_stride = scratch_per;
    a.theta = d_th; a.ntheta = 1; a.status = status; a.out = out1;
    a.px = d_px; a.py = d_py; a.pred_lo = d_plo; a.pred_hi = d_phi; a.pred_leaf = d_sleaf; a.pred_perm = d_perm;
    a.PV = PV; a.PS = PS; a.PVAR = PVAR; a.npred = np;
    a.mean_out = dev ? mean : d_mean;
    a.var_out = dev ? var : d_var;
    HIPCHK(launch_fill_int(status, 1, 0, st));
    HIPCHK(launch_fill(dval, h.nreg, 0.0, st));
    HIPCHK(launch_fill(PV, np * t->WFs, 0.0, st));
    HIPCHK(enqueue_prior(t, pl, a, 1, st));
    if (M > 1 && !pred_chain_tasks.empty()) {
        // the points' whitened rows: the observation chain over the points' arrays
        KArgs b = a;
        b.x = d_px; b.y = d_py; b.obs_lo = d_plo; b.obs_hi = d_phi;
        b.F = PV; b.F_stride = np * t->WFs;
        b.level = M - 1;
        b.tasks = d_pchain;
        b.ntasks = int64_t(pred_chain_tasks.size());
        HIPCHK(launch_chain(b, 1, int(std::min<int64_t>(b.ntasks, 1 << 16)), st));
    }
    a.tasks = d_pleaf;
    a.ntasks = int64_t(pred_leaf_tasks.size());
    HIPCHK(timed(8, M, 0.0, st, [&] { return launch_pred_leaf(a, int(std::min<int64_t>(a.ntasks, nslot)), st); }));
    HIPCHK(enqueue_leaves(t, pl, a, 1, nslot, st));
    for (int m = M - 1; m >= 1; --m) {
        HIPCHK(enqueue_fold(t, pl, a, m, 1, nslot, st));
        a.level = m;
        HIPCHK(timed(9, m, 0.0, st, [&] { return launch_pred_fold(a, st); }));
    }
    HIPCHK(launch_pred_out(a, st));
    if (!dev) {
        HIPCHK(hipMemcpyAsync(mean, d_mean, np * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(var, d_var, np * 8, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(&hstatus, status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hstatus != 0) {
        const int64_t g = hstatus - 1;
        const int lev = region_level(h, g);
        rc = fail(MRA_ENOTPD, "not positive definite: level " + std::to_string(lev) + ", region " +
                                  std::to_string(g - h.lvl_start[lev - 1]));
    }
done:
    (void)hipStreamSynchronize(st);
    for (void* p : {static_cast<void*>(d_th), static_cast<void*>(vst), static_cast<void*>(F), static_cast<void*>(gram),
                    static_cast<void*>(dval), static_cast<void*>(scratch), static_cast<void*>(PV),
                    static_cast<void*>(PS), static_cast<void*>(PVAR), static_cast<void*>(d_px),
                    static_cast<void*>(d_py), static_cast<void*>(d_mean), static_cast<void*>(d_var),
                    static_cast<void*>(out1), static_cast<void*>(status), static_cast<void*>(d_plo),
                    static_cast<void*>(d_phi), static_cast<void*>(d_sleaf), static_cast<void*>(d_perm),
                    static_cast<void*>(d_pleaf), static_cast<void*>(d_pchain)})
        if (p) (void)hipFree(p);
    return rc;
}
