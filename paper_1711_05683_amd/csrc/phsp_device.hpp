// phsp_device.hpp -- per-event device code of the phase-space generator.
//
// One event per lane: counter-based random words, uniforms, an in-register
// sorting network, the invariant masses of the nested subsystems, two-body
// breakup momenta, the weight, isotropic decay angles and the chain of Lorentz
// boosts back to the parent frame (Raubold-Lynch method, arXiv:1711.05683
// sec. 4.2).  Everything here is register-resident; the kernels that include
// this header own the memory traffic (SoA stores) and the reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phsp_sortnet.hpp"

namespace hphsp {

constexpr int kNMax = 10;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplies and xors on a 4-word counter; the 2-word key advances by the Weyl
// increments between rounds.  Key words are wave-uniform, so the key schedule
// runs on the scalar unit.
constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

struct Words4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
        const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ (k0 + (uint32_t)r * kPhiloxWeylA);
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ (k1 + (uint32_t)r * kPhiloxWeylB);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
    }
    return Words4{c0, c1, c2, c3};
}

// Two words -> one uniform on the open 52-bit grid (2x+1) 2^-53, x = the top 52
// bits of (hi:lo).  Built as (1 + x 2^-52) - 1 + 2^-53: every step is exact.
__device__ __forceinline__ double uniform_from_words(uint32_t lo, uint32_t hi) {
    const uint64_t x = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 12;
    const double one_plus = __longlong_as_double((long long)(0x3FF0000000000000ull | x));
    return (one_plus - 1.0) + 0x1p-53;
}

// Per-channel constants, computed once on the host.
struct Channel {
    double M;          // parent mass
    double T;          // M - sum of daughter masses (> 0)
    double C;          // weight constant pi^{N-1} (2T)^{N-2} / (M (N-2)!)
    double half_inv_M; // 1 / (2M)
    double m[kNMax];   // daughter masses
    double S[kNMax];   // prefix sums m_0 + ... + m_i
};

// Parent frame of an event: a pure boost with rapidity vector eta = P/M,
// gamma = E/M, and 1/(gamma+1).
struct Frame {
    double eta[3];
    double gamma;
    double inv_gp1;
};

// Four-momenta of one event's daughters, in registers.
template <int N, typename R>
struct Event {
    R e[N], x[N], y[N], z[N];
};

// Boost of (E, p) by rapidity vector eta (eta = gamma beta):
//   E' = gamma E + eta.p,  p' = p + (eta.p / (gamma + 1) + E) eta.
template <typename R>
__device__ __forceinline__ void boost(R& e, R& x, R& y, R& z, R ex, R ey, R ez, R gamma, R inv_gp1) {
    const R ep = fma(ex, x, fma(ey, y, ez * z));
    const R f = fma(ep, inv_gp1, e);
    e = fma(gamma, e, ep);
    x = fma(f, ex, x);
    y = fma(f, ey, y);
    z = fma(f, ez, z);
}

// The random words of global event g: J Philox blocks, counter (g lo, g hi, j, sid).
template <int N>
struct Draws {
    static constexpr int kUniforms = 3 * N - 4;
    static constexpr int kBlocks = (2 * kUniforms + 3) / 4;
    double u[kUniforms];
};

template <int N>
__device__ __forceinline__ void draw_uniforms(Draws<N>& d, uint32_t k0, uint32_t k1, uint32_t sid,
                                              uint64_t g) {
    const uint32_t glo = (uint32_t)g, ghi = (uint32_t)(g >> 32);
#pragma unroll
    for (int j = 0; j < Draws<N>::kBlocks; ++j) {
        const Words4 w = philox4x32_10(glo, ghi, (uint32_t)j, sid, k0, k1);
        if (2 * j < Draws<N>::kUniforms) d.u[2 * j] = uniform_from_words(w.x, w.y);
        if (2 * j + 1 < Draws<N>::kUniforms) d.u[2 * j + 1] = uniform_from_words(w.z, w.w);
    }
}

// FP64 part shared by both precisions: sorted mass uniforms -> invariant masses
// sigma_i, breakup momenta p_i, 1/sigma_i, and the weight C prod p_i.
template <int N>
struct Levels {
    double p[N - 1];     // breakup momentum of level i (sigma_{i+1} -> sigma_i + m_{i+1})
    double sigma[N];     // invariant mass of daughters {0..i}
    double inv_sigma[N]; // 1 / sigma_i for 1 <= i <= N-2
    double w;            // event weight
};

template <int N>
__device__ __forceinline__ void solve_levels(const Channel& c, Draws<N>& d, Levels<N>& L) {
    // Sorted R_1..R_{N-2}; R_0 = 0 and R_{N-1} = 1 are implicit.
    sortnet_sort<N - 2>(d.u);
    L.sigma[0] = c.m[0];
#pragma unroll
    for (int i = 1; i <= N - 2; ++i) L.sigma[i] = fma(c.T, d.u[i - 1], c.S[i]);
    L.sigma[N - 1] = c.M;
#pragma unroll
    for (int i = 1; i <= N - 2; ++i) L.inv_sigma[i] = 1.0 / L.sigma[i];
    double w = c.C;
#pragma unroll
    for (int i = 0; i <= N - 2; ++i) {
        const double r_hi = (i + 1 <= N - 2) ? d.u[i] : 1.0;
        const double r_lo = (i >= 1) ? d.u[i - 1] : 0.0;
        const double g = c.T * (r_hi - r_lo); // energy released at level i
        const double b = L.sigma[i], m = c.m[i + 1];
        const double q = g * (2.0 * b + 2.0 * m + g) * (g + 2.0 * m) * (2.0 * b + g);
        const double half_inv = (i + 1 <= N - 2) ? 0.5 * L.inv_sigma[i + 1] : c.half_inv_M;
        L.p[i] = sqrt(q) * half_inv;
        w *= L.p[i];
    }
    L.w = w;
}

// Direction of level i from its (theta, phi) uniforms:
// cos(theta) = 2u - 1, sin(theta) = 2 sqrt(u (1-u)), phi = 2 pi v.
template <typename R>
__device__ __forceinline__ void direction(double u, double v, R& nx, R& ny, R& nz);

template <>
__device__ __forceinline__ void direction<double>(double u, double v, double& nx, double& ny,
                                                  double& nz) {
    const double ct = 2.0 * u - 1.0;
    const double st = 2.0 * sqrt(u * (1.0 - u));
    double sp, cp;
    sincospi(2.0 * v, &sp, &cp);
    nx = st * cp;
    ny = st * sp;
    nz = ct;
}

// FP32 direction from the FP64 uniforms.  2u - 1 and u (1 - u) are formed in
// FP64 (exact / one rounding) before the conversion, so directions near the
// poles keep FP32 relative accuracy, and phi's uniform is first reduced to
// [-1/2, 1/2] (exactly) so its conversion error is absolute, not relative to 1.
template <>
__device__ __forceinline__ void direction<float>(double u, double v, float& nx, float& ny, float& nz) {
    const float ct = (float)(2.0 * u - 1.0);
    const float st = 2.0f * sqrtf((float)(u * (1.0 - u)));
    const float r = (float)(v - rint(v));
    float sp, cp;
    sincospif(2.0f * r, &sp, &cp);
    nx = st * cp;
    ny = st * sp;
    nz = ct;
}

// Kinematics in precision R (double: the plain path; float: the mixed path).
// Level 0 puts daughters 0 and 1 back to back in the rest frame of {0,1}; level
// i adds daughter i+1 against {0..i} and boosts daughters 0..i from the rest
// frame of {0..i} into that of {0..i+1}.
template <int N, typename R>
__device__ __forceinline__ void build_event(const Channel& c, const Draws<N>& d, const Levels<N>& L,
                                            Event<N, R>& ev) {
    {
        R nx, ny, nz;
        direction<R>(d.u[N - 2], d.u[N - 1], nx, ny, nz);
        const R p = R(L.p[0]);
        const R m0 = R(c.m[0]), m1 = R(c.m[1]);
        ev.e[1] = sqrt(fma(p, p, m1 * m1));
        ev.x[1] = p * nx;
        ev.y[1] = p * ny;
        ev.z[1] = p * nz;
        ev.e[0] = sqrt(fma(p, p, m0 * m0));
        ev.x[0] = -ev.x[1];
        ev.y[0] = -ev.y[1];
        ev.z[0] = -ev.z[1];
    }
#pragma unroll
    for (int i = 1; i <= N - 2; ++i) {
        R nx, ny, nz;
        direction<R>(d.u[N - 2 + 2 * i], d.u[N - 1 + 2 * i], nx, ny, nz);
        const R p = R(L.p[i]);
        const R mi = R(c.m[i + 1]);
        ev.e[i + 1] = sqrt(fma(p, p, mi * mi));
        ev.x[i + 1] = p * nx;
        ev.y[i + 1] = p * ny;
        ev.z[i + 1] = p * nz;
        const R sig = R(L.sigma[i]);
        const R isig = R(L.inv_sigma[i]);
        const R eta = -(p * isig);
        const R ex = eta * nx, ey = eta * ny, ez = eta * nz;
        const R gamma = sqrt(fma(p, p, sig * sig)) * isig;
        const R inv_gp1 = R(1) / (gamma + R(1));
#pragma unroll
        for (int k = 0; k <= i; ++k)
            boost<R>(ev.e[k], ev.x[k], ev.y[k], ev.z[k], ex, ey, ez, gamma, inv_gp1);
    }
}

template <int N, typename R>
__device__ __forceinline__ void boost_to_lab(Event<N, R>& ev, const Frame& f) {
    const R ex = R(f.eta[0]), ey = R(f.eta[1]), ez = R(f.eta[2]);
    const R gamma = R(f.gamma), inv_gp1 = R(f.inv_gp1);
#pragma unroll
    for (int k = 0; k < N; ++k) boost<R>(ev.e[k], ev.x[k], ev.y[k], ev.z[k], ex, ey, ez, gamma, inv_gp1);
}

} // namespace hphsp
