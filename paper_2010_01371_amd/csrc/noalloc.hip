// mbmd_project_noalloc: the forward projection of mbmd_project for callers
// that cannot allocate device memory.  The geometry tables and the line-prefix
// scratch live in one file-scope device array instead of library allocations.
//
// The array's name is a host-side stand-in in host code: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is passed to the kernels and to copies.  Every call on
// a device shares the device's array, which keeps the tables of the last
// geometry placed there; calls that overlap on one device race.
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace mbmd {
namespace {

constexpr size_t kScratchBytes = MBMD_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) char scratch[kScratchBytes];

// What a device's array holds.
struct DeviceScratch {
    char* ptr = nullptr;            // device address of that device's scratch
    bool have_tables = false;
    std::string key;                // geometry the tables belong to
    GeomTables t;                   // pointers into ptr
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxGpus];

std::string geometry_key(const mbmd_geometry& g) {
    const double f[] = {(double)g.kind, (double)g.nx, (double)g.ny, g.dx, g.dy, (double)g.n_views,
                        g.theta0, g.dtheta, (double)g.n_bins, g.du, g.u_offset, g.dso, g.dsd};
    return std::string(reinterpret_cast<const char*>(f), sizeof(f));
}

}  // namespace
}  // namespace mbmd

using namespace mbmd;

extern "C" int mbmd_project_noalloc(const mbmd_geometry* geom, const float* x_dev, float* sino_dev, int n_mat,
                                    void* stream) {
    (void)hipGetLastError();
    try {
        MBMD_REQUIRE(geom && x_dev && sino_dev, MBMD_ERR_ARG, "NULL argument");
        validate_geometry(*geom);
        MBMD_REQUIRE(n_mat >= 1 && n_mat <= kMaxMat, MBMD_ERR_SHAPE, "n_mat must be in 1..4");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (geom->kind == MBMD_GEOM_IDENTITY) {
            MBMD_HIP(hipMemcpyAsync(sino_dev, x_dev, sizeof(float) * (size_t)n_mat * geom->nx * geom->ny,
                                    hipMemcpyDeviceToDevice, s));
            return MBMD_OK;
        }
        // tables and the prefix scratch for every material count, so that one
        // placement serves all later calls with this geometry
        const size_t need = geometry_bytes(*geom, kMaxMat, 0);
        MBMD_REQUIRE(need <= kScratchBytes, MBMD_ERR_SHAPE,
                     "geometry too large for the allocation-free projector (" + std::to_string(need) +
                         " bytes of tables and scratch, at most " + std::to_string(kScratchBytes) + ")");
        int dev = 0;
        MBMD_HIP(hipGetDevice(&dev));
        MBMD_REQUIRE(dev >= 0 && dev < kMaxGpus, MBMD_ERR_ARG, "device index out of range");
        std::lock_guard<std::mutex> lock(g_mu);
        DeviceScratch& d = g_dev[dev];
        if (d.ptr == nullptr) {
            void* p = nullptr;
            MBMD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            MBMD_REQUIRE(p != nullptr, MBMD_ERR_HIP, "no device address for the projector scratch");
            d.ptr = static_cast<char*>(p);
        }
        const std::string key = geometry_key(*geom);
        if (!d.have_tables || d.key != key) {
            // Another geometry: build its tables on the host and place them.  Work
            // already enqueued on this device may still read the old ones.
            GeomHost h;
            build_geometry_host(*geom, h);
            d.have_tables = false;
            MBMD_HIP(hipDeviceSynchronize());
            place_geometry(*geom, h, d.t, d.ptr, kMaxMat, 0, s);
            MBMD_HIP(hipStreamSynchronize(s));          // h goes out of scope
            d.key = key;
            d.have_tables = true;
        }
        launch_project(d.t, x_dev, sino_dev, n_mat, s);
        return MBMD_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::exception& e) {
        set_error(e.what());
        return MBMD_ERR_HIP;
    } catch (...) {
        set_error("unknown error");
        return MBMD_ERR_HIP;
    }
}
