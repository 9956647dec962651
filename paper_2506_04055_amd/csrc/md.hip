// NVT molecular dynamics on the device: velocity Verlet inside a Nosé–Hoover
// chain thermostat (the ensemble of the paper's MD runs; Methods, "Molecular
// Dynamics Simulations": Nosé–Hoover with a temperature damping time).
//
// One step of length dt is the symmetric splitting
//   C(dt/2)  V(dt/2) X(dt) [F] V(dt/2)  C(dt/2)
// where V/X are the velocity-Verlet kick and drift and C(h) propagates the
// chain of M thermostats {xi_k, v_k} with masses Q_1 = N_f kB T tau^2,
// Q_k = kB T tau^2 (k > 1) over a time h.  Inside C(h) the thermostat forces
//   G_1 = (2 KE - N_f kB T) / Q_1,   G_k = (Q_{k-1} v_{k-1}^2 - kB T) / Q_k
// act on the thermostat velocities in a backward sweep (k = M .. 1, each v_k
// between two factors exp(-h v_{k+1} / 4) and kicked by h G_k / 2), then the
// particle velocities are scaled by exp(-h v_1) and every xi_k advances by
// h v_k, then a forward sweep (k = 1 .. M) repeats the kicks with the new
// kinetic energy.  This is the first-order Trotter factorisation of the chain
// Liouvillian of Martyna, Tuckerman and Klein; the extended energy
//   H = KE + E_pot + sum_k Q_k v_k^2 / 2 + N_f kB T xi_1 + kB T sum_{k>1} xi_k
// is conserved up to the integrator's O(dt^2) error.
//
// The chain state is FP64 on the device and the kinetic energy is a fixed-
// order FP64 reduction, so a step needs no host round trip besides the
// neighbour-list displacement check of the plain step.
#include "../../include/mlp.h"
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace mlp {

constexpr int MAX_CHAIN = 8;
constexpr int KE_BLOCKS = 512;
constexpr double KB_EV = 8.617333262e-5;      // Boltzmann constant, eV / K
constexpr double MVV2E = 103.6426891;         // amu A^2 / fs^2 -> eV

// Device state: [0] KE (eV) after the last scaling, [1] velocity scale of the
// last half step, [2, 2+M) xi, [2+M, 2+2M) v, [2+2M, 2+3M) Q.
struct NvtLayout {
    int M;
    __host__ __device__ int xi(int k) const { return 2 + k; }
    __host__ __device__ int v(int k) const { return 2 + M + k; }
    __host__ __device__ int q(int k) const { return 2 + 2 * M + k; }
    __host__ __device__ int size() const { return 2 + 3 * M; }
};

// Per-block partial sums of m |v|^2 (amu A^2/fs^2), fixed order.
__global__ void __launch_bounds__(256) k_ke_part(const float *__restrict__ vel, const float *__restrict__ inv_mass,
                                                 int n, double *__restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const double m = 1.0 / (double)inv_mass[i];
        const double vx = vel[i], vy = vel[(long)n + i], vz = vel[2L * n + i];
        acc += m * (vx * vx + vy * vy + vz * vz);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Chain propagation over h with the kinetic energy from the partial sums.
__global__ void k_nhc(const double *__restrict__ part, int nparts, double *__restrict__ st, int M, double nf,
                      double kT, double h) {
    __shared__ double sh[KE_BLOCKS];
    for (int i = threadIdx.x; i < KE_BLOCKS; i += blockDim.x) sh[i] = i < nparts ? part[i] : 0.0;
    __syncthreads();
    for (int off = KE_BLOCKS / 2; off > 0; off >>= 1) {
        for (int i = threadIdx.x; i < off; i += blockDim.x) sh[i] += sh[i + off];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const NvtLayout L{M};
    double ke = 0.5 * MVV2E * sh[0];
    double v[MAX_CHAIN], q[MAX_CHAIN];
    for (int k = 0; k < M; k++) {
        v[k] = st[L.v(k)];
        q[k] = st[L.q(k)];
    }
    auto force = [&](int k) { return k == 0 ? (2.0 * ke - nf * kT) / q[0] : (q[k - 1] * v[k - 1] * v[k - 1] - kT) / q[k]; };
    // backward sweep
    v[M - 1] += 0.5 * h * force(M - 1);
    for (int k = M - 2; k >= 0; k--) {
        const double a = exp(-0.25 * h * v[k + 1]);
        v[k] = (v[k] * a + 0.5 * h * force(k)) * a;
    }
    // particles and thermostat positions
    const double s = exp(-h * v[0]);
    ke *= s * s;
    for (int k = 0; k < M; k++) st[L.xi(k)] += h * v[k];
    // forward sweep
    for (int k = 0; k < M - 1; k++) {
        const double a = exp(-0.25 * h * v[k + 1]);
        v[k] = (v[k] * a + 0.5 * h * force(k)) * a;
    }
    v[M - 1] += 0.5 * h * force(M - 1);
    for (int k = 0; k < M; k++) st[L.v(k)] = v[k];
    st[0] = ke;
    st[1] = s;
}

__global__ void k_scale_v(float *__restrict__ vel, long cnt, const double *__restrict__ st) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) vel[i] = (float)((double)vel[i] * st[1]);
}

}  // namespace mlp

using namespace mlp;

struct mlp_nvt {
    int n_dof = 0, M = 0;
    double T = 0, tau = 0;
    double *st = nullptr;     // device chain state (NvtLayout)
    double *part = nullptr;   // device KE partial sums [KE_BLOCKS]
};

namespace mlp {

static int nvt_half(mlp_nvt *t, float *vel, const float *inv_mass, int n, double h, hipStream_t s) {
    const int nb = std::max(1, std::min((n + 255) / 256, KE_BLOCKS));
    k_ke_part<<<nb, 256, 0, s>>>(vel, inv_mass, n, t->part);
    k_nhc<<<1, 64, 0, s>>>(t->part, nb, t->st, t->M, (double)t->n_dof, KB_EV * t->T, h);
    k_scale_v<<<(unsigned)((3L * n + 255) / 256), 256, 0, s>>>(vel, 3L * n, t->st);
    HIP_TRY(hipGetLastError());
    return 0;
}

}  // namespace mlp

extern "C" {

int mlp_nvt_create(int32_t n_dof, double temperature, double tau_fs, int32_t chain, mlp_nvt **out) {
    if (!out) return fail(MLP_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (n_dof < 1 || !(temperature > 0.0) || !(tau_fs > 0.0) || chain < 1 || chain > MAX_CHAIN)
        return fail(MLP_ERR_INVALID_ARG, "need n_dof >= 1, temperature > 0, tau > 0 and 1 <= chain <= 8");
    mlp_nvt *t = new mlp_nvt();
    t->n_dof = n_dof;
    t->M = chain;
    t->T = temperature;
    t->tau = tau_fs;
    const NvtLayout L{chain};
    std::vector<double> h(L.size(), 0.0);
    const double kT = KB_EV * temperature;
    for (int k = 0; k < chain; k++) h[L.q(k)] = (k == 0 ? (double)n_dof : 1.0) * kT * tau_fs * tau_fs;
    h[1] = 1.0;
    if (hipMalloc(&t->st, sizeof(double) * L.size()) != hipSuccess ||
        hipMalloc(&t->part, sizeof(double) * KE_BLOCKS) != hipSuccess) {
        (void)hipGetLastError();
        if (t->st) hipFree(t->st);
        delete t;
        return fail(MLP_ERR_OOM, "thermostat allocation failed");
    }
    if (hipMemcpy(t->st, h.data(), sizeof(double) * L.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(t->st);
        hipFree(t->part);
        delete t;
        return fail(MLP_ERR_DEVICE, "thermostat upload failed");
    }
    *out = t;
    return MLP_OK;
}

int mlp_nvt_destroy(mlp_nvt *t) {
    if (!t) return MLP_OK;
    if (t->st) hipFree(t->st);
    if (t->part) hipFree(t->part);
    delete t;
    return MLP_OK;
}

int mlp_nvt_read(mlp_nvt *t, double *xi, double *vxi, double *thermostat_energy, double *kinetic, void *stream) {
    if (!t) return fail(MLP_ERR_INVALID_ARG, "null thermostat");
    const NvtLayout L{t->M};
    std::vector<double> h(L.size());
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(h.data(), t->st, sizeof(double) * L.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MLP_ERR_DEVICE, "thermostat readback failed");
    const double kT = KB_EV * t->T;
    double eth = 0.0;
    for (int k = 0; k < t->M; k++) {
        if (xi) xi[k] = h[L.xi(k)];
        if (vxi) vxi[k] = h[L.v(k)];
        eth += 0.5 * h[L.q(k)] * h[L.v(k)] * h[L.v(k)] + (k == 0 ? (double)t->n_dof : 1.0) * kT * h[L.xi(k)];
    }
    if (thermostat_energy) *thermostat_energy = eth;
    if (kinetic) *kinetic = h[0];
    return MLP_OK;
}

int mlp_md_step_nvt(mlp_model *m, mlp_nbr *g, mlp_nvt *t, float *pos, float *vel, float *forces,
                    const float *inv_mass, const int32_t *species, int32_t n, const double box[3], float skin,
                    float dt, void *stream, double *energy, int32_t *rebuilt) {
    if (!t) return fail(MLP_ERR_INVALID_ARG, "null thermostat");
    if (!vel || !inv_mass || n <= 0) return fail(MLP_ERR_INVALID_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = nvt_half(t, vel, inv_mass, n, 0.5 * (double)dt, s))) return rc;
    if ((rc = mlp_md_step(m, g, pos, vel, forces, inv_mass, species, n, box, skin, dt, stream, energy, rebuilt)))
        return rc;
    return nvt_half(t, vel, inv_mass, n, 0.5 * (double)dt, s);
}

}  // extern "C"
