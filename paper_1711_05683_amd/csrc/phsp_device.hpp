// phsp_device.hpp -- per-event device code of the phase-space generator.
//
// One event per lane: counter-based random words, uniforms, an in-register
// sorting network, the invariant masses of the nested subsystems, two-body
// breakup momenta, the weight, isotropic decay angles and the chain of Lorentz
// boosts back to the parent frame (Raubold-Lynch method, arXiv:1711.05683
// sec. 4.2).  Everything here is register-resident; the kernels that include
// this header own the memory traffic (SoA stores) and the reductions.
//
// Uniform k of an event is built from words 2k and 2k+1 of its Philox stream,
// i.e. from half k&1 of call k>>1.  The N-2 mass uniforms come first; the
// (theta, phi) pair of level i are uniforms N-2+2i and N-1+2i, drawn only when
// that level is built (so integrate-only launches never draw angles, and only
// two angle uniforms are live at a time).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "phsp_sortnet.hpp"

namespace hphsp {

constexpr int kNMax = 10;
constexpr int kTrigSize = 256; // entries of the (cos, sin)(2 pi k / 256) table

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
        // three-input xor in one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0 + (uint32_t)r * kPhiloxWeylA, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1 + (uint32_t)r * kPhiloxWeylB, 0x96);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
    }
    return Words4{c0, c1, c2, c3};
}

// Two words -> one uniform on the open 52-bit grid (2x+1) 2^-53, x = the top 52
// bits of (hi:lo).  Built as (1 + x 2^-52) - (1 - 2^-53): both operands lie
// within a factor of two of each other, so the one subtraction is exact
// (Sterbenz) and gives (2x+1) 2^-53 directly.
__device__ __forceinline__ double uniform_from_words(uint32_t lo, uint32_t hi) {
    const uint64_t x = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 12;
    const double one_plus = __longlong_as_double((long long)(0x3FF0000000000000ull | x));
    return one_plus - (1.0 - 0x1p-53);
}

// Counter state of one event's stream: call j uses counter (g lo, g hi, j, sid).
struct EventRng {
    uint32_t glo, ghi, sid, k0, k1;
    __device__ __forceinline__ void call(uint32_t j, double& a, double& b) const {
        const Words4 w = philox4x32_10(glo, ghi, j, sid, k0, k1);
        a = uniform_from_words(w.x, w.y);
        b = uniform_from_words(w.z, w.w);
    }
};

// Reciprocal to full double precision: the hardware estimate refined by two
// Newton-Raphson steps (each squares the relative error).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Square root of x for x = 0 or finite x >= 2^-767: the hardware
// reciprocal-square-root estimate r, one Goldschmidt step on (g, h) = (x r, r/2)
// and two Newton corrections g += (x - g^2) h.  For these arguments this is the
// same sequence, and the same result, as the general double square root,
// without its rescaling of tiny arguments and its special cases; x = 0 (where
// r is infinite) gives 0 because the estimate is capped at 2^500.  The
// generator's arguments are pdk products and u(1-u) with u >= 2^-53.
__device__ __forceinline__ double sqrt_pos(double x) {
    const double r = fmin(__builtin_amdgcn_rsq(x), 0x1p+500);
    double g = x * r;
    double h = 0.5 * r;
    const double e = fma(-h, g, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
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

// Mass uniforms of one event (sorted in place by event_levels).  For odd N the
// last mass call also yields level 0's theta uniform, kept in `carry`.
template <int N>
struct MassDraws {
    static constexpr int kMass = N - 2;
    double u[kMass > 0 ? kMass : 1];
    double carry;
};

template <int N>
__device__ __forceinline__ void draw_masses(MassDraws<N>& d, const EventRng& rng) {
#pragma unroll
    for (int j = 0; 2 * j + 1 < N - 2; ++j) rng.call((uint32_t)j, d.u[2 * j], d.u[2 * j + 1]);
    if constexpr ((N - 2) % 2 == 1) {
        double a, b;
        rng.call((uint32_t)((N - 3) / 2), a, b);
        d.u[N - 3] = a;
        d.carry = b;
    } else {
        d.carry = 0.0;
    }
}

// (theta, phi) uniforms of level i, drawn on demand.  For even N they are both
// halves of call (N-2)/2 + i; for odd N, theta is the carried second half of the
// previous call and phi the first half of call (N-1)/2 + i.
template <int N>
__device__ __forceinline__ void draw_angles(const EventRng& rng, int i, double& carry, double& ut, double& up) {
    if constexpr (N % 2 == 0) {
        rng.call((uint32_t)((N - 2) / 2 + i), ut, up);
    } else {
        ut = carry;
        rng.call((uint32_t)((N - 1) / 2 + i), up, carry);
    }
}

// sin and cos of 2 pi v for v in (0, 1): v = k/256 + f/256 with k = rint(256 v)
// and |f| <= 1/2 (both exact); the table holds (cos, sin)(2 pi k/256) and short
// Taylor series give sin d and cos d - 1 for d = 2 pi f/256, |d| <= pi/256
// (truncation below 1e-20), combined by the angle-addition formulas.
__device__ __forceinline__ void sincos_2pi_table(double v, const double2* tab, double& s, double& c) {
    const double x = v * (double)kTrigSize;
    const double k = rint(x);
    const double d = (x - k) * 0.02454369260617026; // 2 pi / 256
    const double d2 = d * d;
    const double sd = fma(d * d2, fma(d2, fma(d2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), d);
    const double cm1 = d2 * fma(d2, fma(d2, -1.0 / 720.0, 1.0 / 24.0), -0.5);
    const double2 t = tab[((int)k) & (kTrigSize - 1)];
    s = fma(t.y, cm1, fma(t.x, sd, t.y));
    c = fma(t.x, cm1, fma(-t.y, sd, t.x));
}

// Momentum p n of a level from its (theta, phi) uniforms, n the direction with
// cos(theta) = 2u - 1, sin(theta) = 2 sqrt(u (1-u)), phi = 2 pi v; the
// transverse part is (p sin(theta)) (cos(phi), sin(phi)).
__device__ __forceinline__ void level_momentum(double p, double u, double v, const double2* tab, double& px,
                                               double& py, double& pz) {
    const double ct = 2.0 * u - 1.0;
    const double st = 2.0 * sqrt_pos(u * (1.0 - u));
    double sp, cp;
    sincos_2pi_table(v, tab, sp, cp);
    const double pt = p * st;
    px = pt * cp;
    py = pt * sp;
    pz = p * ct;
}

// Energies of the two bodies of a level in the rest frame of hi = lo + m + g:
//   E(m) = (hi^2 + m^2 - lo^2) / (2 hi) = ((m + g)(hi + lo) + m^2) h,  h = 1/(2 hi),
// and E(lo) likewise with m and lo exchanged; every term is non-negative, so
// nothing cancels.
__device__ __forceinline__ double level_energy(double m, double lo, double g, double hi, double h) {
    return fma(m + g, hi + lo, m * m) * h;
}

// All two-body levels of one event, in one pass.  The weight (always FP64) is
// C prod_i p_i with the invariant masses sigma_i = S_i + T R_i of the sorted
// mass uniforms, the energy released g_i = T (R_{i+1} - R_i) and the breakup
// momentum p_i of sigma_{i+1} -> sigma_i + m_{i+1}.  With KIN, the kinematics of
// the level follow at once, in FP64 for every output precision: level 0 puts
// daughters 0 and 1 back to back in the rest frame of {0,1}; level i adds
// daughter i+1 against {0..i} and boosts daughters 0..i from the rest frame of
// {0..i} into that of {0..i+1}.  Only the current level's quantities are live,
// besides the sorted uniforms and the momenta.
//
// The momenta stay FP64 between boosts even when the outputs are FP32: a light
// daughter emitted nearly backwards to a boost of large gamma ends up with a lab
// energy of order E/gamma, and its lab components move by about gamma times any
// relative error in its rest-frame direction.  Rounding the vectors to FP32
// between boosts (a direction error of 2^-24) therefore costs up to gamma * 6e-8
// of the daughter's energy, which for massless daughters (where gamma reaches
// 1e3 and beyond) exceeds 1e-5; rounding once at the store costs 2^-24.
template <int N, bool KIN>
__device__ __forceinline__ double event_levels(const Channel& c, const EventRng& rng, MassDraws<N>& d,
                                               const double2* tab, Event<N, double>& ev) {
    using R = double;
    sortnet_sort<N - 2>(d.u); // R_1..R_{N-2}; R_0 = 0 and R_{N-1} = 1 are implicit
    double carry = d.carry;
    double w = c.C;
    double sig_lo = c.m[0]; // sigma_i
    double inv_lo = 0.0;    // 1 / sigma_i (i >= 1)
#pragma unroll
    for (int i = 0; i <= N - 2; ++i) {
        constexpr int kTop = N - 2;
        const bool inner = i < kTop; // sigma_{i+1} is an inner subsystem, not the parent
        const double r_hi = inner ? d.u[i] : 1.0;
        const double r_lo = (i >= 1) ? d.u[i - 1] : 0.0;
        const double sig_hi = inner ? fma(c.T, r_hi, c.S[i + 1]) : c.M;
        const double inv_hi = inner ? recip(sig_hi) : 0.0;
        const double h = inner ? 0.5 * inv_hi : c.half_inv_M; // 1 / (2 sigma_{i+1})
        const double g = c.T * (r_hi - r_lo);
        const double m = c.m[i + 1];
        const double q = g * (2.0 * sig_lo + 2.0 * m + g) * (g + 2.0 * m) * (2.0 * sig_lo + g);
        const double pd = sqrt_pos(q) * h;
        w *= pd;
        if constexpr (KIN) {
            double ut, up;
            draw_angles<N>(rng, i, carry, ut, up);
            level_momentum(pd, ut, up, tab, ev.x[i + 1], ev.y[i + 1], ev.z[i + 1]);
            // Per-level scalars from the gap formulas: no square roots, nothing
            // cancels.
            if (i == 0) {
                ev.e[1] = level_energy(m, sig_lo, g, sig_hi, h);
                ev.e[0] = level_energy(sig_lo, m, g, sig_hi, h);
                ev.x[0] = -ev.x[1];
                ev.y[0] = -ev.y[1];
                ev.z[0] = -ev.z[1];
            } else {
                ev.e[i + 1] = level_energy(m, sig_lo, g, sig_hi, h);
                const double esys = level_energy(sig_lo, m, g, sig_hi, h); // energy of {0..i}
                const R gamma = esys * inv_lo;
                const R inv_gp1 = sig_lo * recip(esys + sig_lo); // 1/(gamma+1) = sigma / (E + sigma)
                // eta = -(p_i / sigma_i) n: the new daughter's momentum scaled
                const R ex = ev.x[i + 1] * -inv_lo, ey = ev.y[i + 1] * -inv_lo, ez = ev.z[i + 1] * -inv_lo;
#pragma unroll
                for (int k = 0; k <= i; ++k)
                    boost<R>(ev.e[k], ev.x[k], ev.y[k], ev.z[k], ex, ey, ez, gamma, inv_gp1);
            }
        }
        sig_lo = sig_hi;
        inv_lo = inv_hi;
    }
    return w;
}

template <int N>
__device__ __forceinline__ void boost_to_lab(Event<N, double>& ev, const Frame& f) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        boost<double>(ev.e[k], ev.x[k], ev.y[k], ev.z[k], f.eta[0], f.eta[1], f.eta[2], f.gamma, f.inv_gp1);
}

// The block's copy of the (cos, sin) table: filled once per block from the
// library's device table (block size >= kTrigSize), then read per lane.
__device__ __forceinline__ void load_trig(double2* lds, const double2* global) {
    if (threadIdx.x < kTrigSize) lds[threadIdx.x] = global[threadIdx.x];
    __syncthreads();
}

} // namespace hphsp
