// harness.hip -- client-side work of the serving harness (not part of the QED library).
//
// The served form runs simulated PIC clients whose particles need a momentum push before every
// QED step (the step's beyond-LCFA form needs the momentum before and after the push).  This
// file holds that client push as one kernel, so that a client's tick costs one launch instead
// of a dozen framework operations.  It is built into its own shared library,
// libsfq_harness.so, which the serving harness loads; the QED library does not use it.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

// Lorentz-force kick of charge -1 in the plane wave E = a cos(phi + t) y, B = a cos(phi + t) z:
//   dp/dt = -(E + v x B) = (-v_y a c, -(1 - v_x) a c, 0),  c = cos(phi + t),  v = p / gamma,
// explicit in time; p_prev receives the momentum before the kick.
__global__ __launch_bounds__(256) void push_kernel(size_t n, double* __restrict__ px,
                                                   double* __restrict__ py,
                                                   const double* __restrict__ pz,
                                                   double* __restrict__ qx,
                                                   double* __restrict__ qy,
                                                   double* __restrict__ qz,
                                                   const double* __restrict__ a,
                                                   const double* __restrict__ phi, double t,
                                                   double dt)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double x = px[i], y = py[i], z = pz[i];
        qx[i] = x;
        qy[i] = y;
        qz[i] = z;
        const double amp = a[i] * cos(phi[i] + t);
        const double ginv = 1.0 / sqrt(1.0 + (x * x + y * y + z * z));
        px[i] = x - dt * (y * ginv) * amp;
        py[i] = y - dt * (1.0 - x * ginv) * amp;
    }
}

}  // namespace

extern "C" {

// Pushes n electrons (device arrays of n doubles each; p updated in place, p_prev written) at
// field phase offset t with time step dt, on `stream`.  Returns 0, or the HIP error code.
int harness_push_plane_wave(size_t n, double* px, double* py, const double* pz, double* px_prev,
                            double* py_prev, double* pz_prev, const double* a, const double* phi,
                            double t, double dt, void* stream)
{
    if (n == 0) return 0;
    const size_t blocks = (n + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(push_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, n, px, py, pz,
                       px_prev, py_prev, pz_prev, a, phi, t, dt);
    return (int)hipGetLastError();
}

}  // extern "C"
