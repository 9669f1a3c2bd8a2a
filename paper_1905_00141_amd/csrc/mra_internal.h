// Internal declarations shared by the host-side tree builder and the HIP
// library.  Not part of the ABI.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace mra {

enum FoldForm : int8_t { FOLD_FACTOR = 0, FOLD_GRAM = 1 };

constexpr int MAXL_TREE = 16;  // most levels a partition may have

// Host-side description of the partition (Sec. 1.2) plus the execution plan
// derived from it.  Regions are numbered in level order; the children of
// region k at level m are J*k .. J*k+J-1 at level m+1, so every region's
// observations are one contiguous range of the leaf-grouped order.
struct HostTree {
    int J = 4, M = 1, r = 1, nx = 1, ny = 1, rhat = 1, P = 16;
    double offset = 0.0;
    int64_t n_in = 0, n_nan = 0, n_elim = 0, n_used = 0, n_dup = 0;
    int64_t nreg = 0, nleaf = 0;
    std::vector<int64_t> lvl_start;  // M + 1 entries
    std::vector<double> box;         // nreg * 4 (xlo, xhi, ylo, yhi)
    std::vector<int64_t> obs_lo;     // nreg + 0: first observation of each region's subtree
    std::vector<int64_t> obs_hi;     // one past the last
    std::vector<double> x, y, z;     // used observations, grouped by leaf
    std::vector<int64_t> orig;       // input index of each used observation
};

// Builds the partition on the GPU from device-resident x, y, z (no duplicate
// elimination); the grouped observations and their input indices are
// returned in new device arrays, t.x / t.y / t.z / t.orig stay empty.
int build_device_tree(const double* x, const double* y, const double* z, int64_t n, int J, int r, int M,
                      double offset, const double* domain4, HostTree& t, double** ox, double** oy, double** oz,
                      int64_t** oorig, std::string& err);

// Builds the partition on the host.  Returns an MRA_* status, message in err.
int build_host_tree(const double* x, const double* y, const double* z, int64_t n, int J, int r,
                    int M, double offset, uint32_t flags, const double* domain4, HostTree& t, std::string& err);

}  // namespace mra

namespace mra {
// Error reporting and pointer classification shared by the library's entry
// points: fail() records the thread-local message of mra_last_error.
int fail(int code, const std::string& msg);
bool is_device_ptr(const void* p);
int check_device();

// Leaf (global level-order index) of each location by descent from the root;
// MRA_EDOMAIN for a location outside the root region.
int locate_leaves(const HostTree& t, const double* x, const double* y, int64_t n, std::vector<int64_t>& leaf,
                  std::string& err);
}  // namespace mra
