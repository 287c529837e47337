// rpy_noalloc.hip -- rpy_forces_noalloc: the spring and excluded-volume
// forces of rpy_forces without a context, for callers that cannot allocate
// device memory (code under stream capture, tight stepping loops).  The
// kernels are those of rpy_forces; their scratch (the wrapped positions, the
// cell list and its cursors, the non-finite flag) lives in one file-scope
// device array instead of context buffers.
#include <math.h>

#include <mutex>

#include "rpy_internal.h"

using namespace rpy;

namespace {

constexpr int NA_MAX_BEADS = 65536;   // largest N accepted
constexpr int NA_MAX_CELLS = 64;      // cells per side of the cell list (as rpy_forces)
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t NA_RT_OFF = 0;                                             // double [N][3]
constexpr size_t NA_START_OFF = align256(sizeof(double) * 3 * NA_MAX_BEADS); // int [2 nc^3 + 1]
constexpr size_t NA_BEADS_OFF =
    NA_START_OFF + align256(sizeof(int) * (2 * (size_t)NA_MAX_CELLS * NA_MAX_CELLS * NA_MAX_CELLS + 1));
constexpr size_t NA_FLAG_OFF = NA_BEADS_OFF + align256(sizeof(int) * NA_MAX_BEADS);  // int [1]
constexpr size_t NA_BYTES = NA_FLAG_OFF + 256;   // 3.9 MB

}  // namespace

// The scratch of every call on a device.  Its name is a host-side stand-in:
// host code uses only the device address taken below.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char *g_scratch[NA_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_of_current_device(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "rpy_forces_noalloc: hipGetDevice");
    if (dev < 0 || dev >= NA_MAX_DEVICES) {
        set_error("rpy_forces_noalloc: device index beyond 63");
        return RPY_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_error(e, "rpy_forces_noalloc: hipGetSymbolAddress");
        g_scratch[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch[dev];
    return RPY_OK;
}

}  // namespace

extern "C" int rpy_forces_noalloc(int n_beads, int n_chains, int beads_per_chain, double box_l,
                                  const double *pos, double zstar, double dstar, double rcut,
                                  double *out, void *stream)
{
    if (!pos || !out || n_beads <= 0 || n_chains <= 0 || beads_per_chain <= 0 ||
        (int64_t)n_chains * beads_per_chain != n_beads || !(box_l > 0) || !isfinite(box_l)) {
        set_error("rpy_forces_noalloc: invalid sizes, box or null pointers");
        return RPY_EINVAL;
    }
    if (n_beads > NA_MAX_BEADS) {
        set_error("rpy_forces_noalloc: n_beads beyond 65536, the size of its scratch");
        return RPY_EINVAL;
    }
    if (zstar < 0 || !isfinite(zstar) ||
        (zstar > 0 && (!(dstar > 0) || !isfinite(dstar) || !(rcut > 0) || !(rcut < 0.5 * box_l)))) {
        set_error("rpy_forces_noalloc: excluded volume needs d* > 0 and 0 < rcut < L/2");
        return RPY_EINVAL;
    }
    unsigned char *base = nullptr;
    int rc = scratch_of_current_device(&base);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx c;
    c.N = n_beads;
    c.n3 = 3 * n_beads;
    c.nchains = n_chains;
    c.bpc = beads_per_chain;
    c.L = box_l;
    c.ncell = 0;
    c.flags = reinterpret_cast<int *>(base + NA_FLAG_OFF);
    c.cell_start = reinterpret_cast<int *>(base + NA_START_OFF);
    c.cell_beads = reinterpret_cast<int *>(base + NA_BEADS_OFF);
    double *rt = reinterpret_cast<double *>(base + NA_RT_OFF);
    launch_spring_forces(c, pos, out, s);
    if (zstar > 0) {
        // as rpy_forces: cells of side >= rcut when there are at least 3 per
        // side, else all pairs; the cell counts are cleared by a kernel of
        // the cell list itself, the flag is only written
        const int nc = (int)floor(box_l / rcut);
        c.ncell = nc >= 3 ? (nc > NA_MAX_CELLS ? NA_MAX_CELLS : nc) : 0;
        launch_wrap_positions(c, pos, rt, s);
        launch_cell_list(c, rt, rcut, s);
        launch_ev_forces(c, rt, zstar, dstar, rcut, out, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "rpy_forces_noalloc");
    return RPY_OK;
}
