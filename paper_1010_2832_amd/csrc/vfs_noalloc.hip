// Allocation-free entry point: the liquid volume fractions W_L of one sample
// set (Section 5, Figs. 3-4) straight from a nodal liquid level set, with no
// context and no device allocation.  Its work space -- the sub-cell liquid and
// fluid fractions and the padded weight arrays the fraction kernels write --
// lives in one file-scope device array, `scratch`, of fixed size.  The kernels
// and their operation order are those of vfs_assemble, so the result is
// bit-identical to vfs_get_weights(ctx, set, VFS_WEIGHT_LIQUID, out) on a
// context assembled from the same level set.
#include <cmath>
#include <mutex>
#include <string>

#include "vfs_internal.h"

using namespace vfs;

static constexpr long long kScratchDoubles = 96LL * 1024 * 1024 / 8;   // 96 MiB

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: it passes the per-device pointer from
// hipGetSymbolAddress instead.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// errors are reported through vfs_last_error(NULL)
int nfail(int code, const std::string& m) { return fail_global(code, m); }

// Device address of `scratch` on the current device, looked up once per device.
int scratch_ptr(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return nfail(VFS_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return nfail(VFS_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return nfail(VFS_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return VFS_OK;
}

// bytes of work space a grid needs: sub-cell fractions (two level sets) and
// padded liquid and fluid weights of every set; -1 for invalid sizes
long long work_bytes(int dim, int nx, int ny, int nz) {
    if ((dim != 2 && dim != 3) || nx < 1 || ny < 1 || (dim == 3 && nz < 1)) return -1;
    if (nx > 16384 || ny > 16384 || (dim == 3 && nz > 2048)) return -1;
    const Geo g = make_geo(dim, nx, ny, nz, 1.0);
    const long long sub = (dim == 2 ? 4LL : 8LL) * nx * ny * (dim == 3 ? nz : 1);
    return (2 * sub + 2LL * g.nsets() * g.NP) * 8;
}

}  // namespace

extern "C" {

int vfs_liquid_weights_noalloc(int dim, int nx, int ny, int nz, double w_min,
                               const double* phi_liquid, int set, double* out, void* hip_stream) {
    const long long need = work_bytes(dim, nx, ny, nz);
    if (need < 0) return nfail(VFS_EINVAL, "dim must be 2 or 3 and sizes in range");
    if (need > kScratchDoubles * 8)
        return nfail(VFS_EINVAL, "grid too large for the fixed work space (" +
                                     std::to_string(need) + " bytes needed, " +
                                     std::to_string(kScratchDoubles * 8) + " available)");
    if (!phi_liquid || !out) return nfail(VFS_EINVAL, "NULL level set or output");
    if (!(w_min >= 0.0) || !(w_min < 0.5)) return nfail(VFS_EINVAL, "w_min must be in [0,0.5)");
    const int nsets = dim == 2 ? 4 : 7;
    // public set numbers: 2D cell, x faces, y faces, nodes (VFS_SET_NODE);
    // 3D the seven sets in their order
    int internal;
    if (dim == 2) {
        if (set == VFS_SET_CELL || set == VFS_SET_FACE_X || set == VFS_SET_FACE_Y)
            internal = set;
        else if (set == VFS_SET_NODE)
            internal = 3;
        else
            return nfail(VFS_EINVAL, "bad sample set for 2D");
    } else {
        if (set < 0 || set >= nsets) return nfail(VFS_EINVAL, "bad sample set for 3D");
        internal = set;
    }
    double* base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    const Geo g = make_geo(dim, nx, ny, nz, 1.0);
    const long long sub = (dim == 2 ? 4LL : 8LL) * nx * ny * (dim == 3 ? nz : 1);
    double* thL = base;
    double* thF = thL + sub;
    double* WL = thF + sub;
    double* WF = WL + (long long)nsets * g.NP;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    // the array keeps the previous call's contents: the weight kernels write
    // every valid entry, and the padding is cleared so the padded layout holds
    // zeros outside each set's range as everywhere else in the library
    launch_fill(WL, 2LL * nsets * g.NP, 0.0, s);
    launch_subcell_fractions(g, phi_liquid, thL, false, s);
    launch_fill(thF, sub, 1.0, s);
    launch_weights(g, thL, thF, w_min, WL, WF, s);
    int shp[3];
    set_shape(g, internal, shp);
    launch_unpack(g, shp, WL + (long long)internal * g.NP, out, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nfail(VFS_EHIP, std::string("launch: ") + hipGetErrorString(e));
    return VFS_OK;
}

}  // extern "C"
