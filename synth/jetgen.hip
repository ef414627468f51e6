// jetgen.hip -- device filler for the seeded jet-like epoch stacks.
//
// Input generator only: it writes emissivity and velocity fields in the
// caller's layout (j [M][nz][ny][nx], beta [M][nz][ny][nx][3], float32) from
// parameters drawn on the host (synth/__init__.py).  It contains no step of
// the rendering method and is shared by the tests and the bench alone.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

struct JetParams {
    int nx, ny, nz;
    int n_modes, n_knots;
    float gamma_spine, r_jet;
    float knot_beta, knot_radius, knot_sigma, knot_amp;
    float turb_speed, outside;
    float k[64 * 3];
    float phase[64];
    float knot_z0[16];
    int z_begin, z_count;  // fill only the z-slab [z_begin, z_begin + z_count) of the domain
};

__global__ void __launch_bounds__(256) jet_fill_kernel(JetParams p, double t, float *__restrict__ j,
                                                       float *__restrict__ beta) {
    const long long ncell = (long long)p.nx * p.ny * p.z_count;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        int ix = (int)(c % p.nx);
        int iy = (int)((c / p.nx) % p.ny);
        int iz = p.z_begin + (int)(c / ((long long)p.nx * p.ny));
        float x = ix + 0.5f, y = iy + 0.5f, z = iz + 0.5f;
        float rx = x - 0.5f * p.nx, ry = y - 0.5f * p.ny;
        float r = sqrtf(rx * rx + ry * ry);
        // turbulence: unit-variance Gaussian field advected along +z
        float za = (float)((double)z - (double)p.turb_speed * t);
        float g = 0.f;
        for (int q = 0; q < p.n_modes; q++)
            g += cosf(p.k[3 * q] * x + p.k[3 * q + 1] * y + p.k[3 * q + 2] * za + p.phase[q]);
        g *= sqrtf(2.0f / (float)p.n_modes);
        float rho = expf(0.5f * g - 0.125f);
        bool in_jet = r <= p.r_jet;
        float jv = powf(rho, 1.5f) * (in_jet ? 1.0f : p.outside);
        // knots on the axis, periodic in z
        float boost = 1.0f;
        bool in_knot = false;
        for (int q = 0; q < p.n_knots; q++) {
            double zk = fmod((double)p.knot_z0[q] + (double)p.knot_beta * t, (double)p.nz);
            if (zk < 0) zk += p.nz;
            float dz = (float)((double)z - zk);
            dz -= p.nz * rintf(dz / p.nz);
            float d2 = rx * rx + ry * ry + dz * dz;
            boost += p.knot_amp * expf(-d2 / (2.0f * p.knot_sigma * p.knot_sigma));
            if (d2 <= p.knot_radius * p.knot_radius) in_knot = true;
        }
        jv *= boost;
        float bz = 0.f;
        if (in_jet) {
            float f = r / p.r_jet;
            float gam = 1.2f + (p.gamma_spine - 1.2f) * (1.0f - f * f);
            bz = (float)sqrt(1.0 - 1.0 / ((double)gam * gam));
        }
        if (in_knot) bz = p.knot_beta;
        j[c] = jv;
        beta[3 * c] = 0.f;
        beta[3 * c + 1] = 0.f;
        beta[3 * c + 2] = bz;
    }
}

extern "C" int synth_jet_fill(const JetParams *p, int n_epochs, const double *times, float *j,
                              float *beta, void *stream) {
    if (!p || !times || !j || !beta || n_epochs < 1 || p->nx < 1 || p->ny < 1 || p->nz < 1 ||
        p->n_modes < 1 || p->n_modes > 64 || p->n_knots < 0 || p->n_knots > 16 ||
        p->z_begin < 0 || p->z_count < 1 || p->z_begin + p->z_count > p->nz)
        return -1;
    const long long ncell = (long long)p->nx * p->ny * p->z_count;
    long long blocks = (ncell + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipStream_t s = (hipStream_t)stream;
    for (int m = 0; m < n_epochs; m++) {
        hipLaunchKernelGGL(jet_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, *p, times[m],
                           j + (size_t)m * ncell, beta + (size_t)m * ncell * 3);
        if (hipGetLastError() != hipSuccess) return -2;
    }
    return 0;
}
