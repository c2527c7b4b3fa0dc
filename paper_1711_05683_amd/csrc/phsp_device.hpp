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
// two angle uniforms are live at a time).  The levels are built from the top
// down, and each daughter is handed on as soon as it is final, so a kernel
// holds one subsystem's four-momentum rather than all N daughters.
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

// (theta, phi) uniforms of level i, drawn on demand from the top level down.
// For even N they are both halves of call (N-2)/2 + i.  For odd N, call
// c_j = (N-1)/2 + j holds phi_j (first half) and theta_{j+1} (second half), and
// theta_0 is the second half of the last mass call (MassDraws::carry): the top
// level draws c_{N-2} (phi; its second half is unused) and c_{N-3} (theta), every
// lower level i >= 1 draws c_{i-1} for its theta and keeps that call's phi for
// level i-1 in `phi_next`, and level 0 draws nothing.
template <int N>
__device__ __forceinline__ void draw_angles_down(const EventRng& rng, int i, double theta0, double& phi_next,
                                                 double& ut, double& up) {
    if constexpr (N % 2 == 0) {
        rng.call((uint32_t)((N - 2) / 2 + i), ut, up);
    } else {
        if (i == N - 2) {
            double unused;
            rng.call((uint32_t)((N - 1) / 2 + i), up, unused);
        } else {
            up = phi_next;
        }
        if (i >= 1)
            rng.call((uint32_t)((N - 1) / 2 + i - 1), phi_next, ut);
        else
            ut = theta0;
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

// All two-body levels of one event, in one pass from the top level down.  The
// weight (always FP64) is C prod_i p_i with the invariant masses
// sigma_i = S_i + T R_i of the sorted mass uniforms, the energy released
// g_i = T (R_{i+1} - R_i) and the breakup momentum p_i of
// sigma_{i+1} -> sigma_i + m_{i+1}; its factors are multiplied top level first
// (equal to the product in any order up to rounding).  With KIN, level i splits
// the subsystem {0..i+1}, whose four-momentum P in the parent's rest frame the
// level above produced (the parent itself at the top), into daughter i+1 and
// {0..i}, back to back along the level's direction in the rest frame of
// {0..i+1}, and boosts both into the parent's rest frame with eta = P/sigma_{i+1},
// gamma = P_E/sigma_{i+1}, 1/(gamma+1) = sigma_{i+1}/(P_E + sigma_{i+1}) (no boost
// at the top).  `emit(k, e, x, y, z)` then receives daughter k = i+1, final; at
// level 0 the remaining subsystem is daughter 0 and is emitted too.  Energies in
// the subsystem's rest frame come from the gap formulas (no square roots,
// nothing cancels).  Everything stays FP64 whatever the output precision: a
// light daughter emitted against a boost of large gamma ends up with an energy
// of order E/gamma, and its components move by about gamma times any relative
// error in its rest-frame direction, so rounding to FP32 before the last boost
// would cost up to gamma * 6e-8 of its energy (beyond 1e-5 for massless
// daughters); rounding once at the store costs 2^-24.
template <int N, bool KIN, class Emit>
__device__ __forceinline__ double event_levels(const Channel& c, const EventRng& rng, MassDraws<N>& d,
                                               const double2* tab, Emit&& emit) {
    sortnet_sort<N - 2>(d.u); // R_1..R_{N-2}; R_0 = 0 and R_{N-1} = 1 are implicit
    double w = c.C;
    double sig_hi = c.M;  // sigma_{i+1}
    double inv_hi = 0.0;  // 1 / sigma_{i+1} (inner subsystems)
    double pe = c.M, px = 0.0, py = 0.0, pz = 0.0; // {0..i+1} in the parent's rest frame
    double phi_next = 0.0;
#pragma unroll
    for (int i = N - 2; i >= 0; --i) {
        const bool top = i == N - 2;
        const double r_hi = top ? 1.0 : d.u[i];
        const double r_lo = (i >= 1) ? d.u[i - 1] : 0.0;
        const double sig_lo = (i >= 1) ? fma(c.T, r_lo, c.S[i]) : c.m[0];
        const double inv_lo = (i >= 1) ? recip(sig_lo) : 0.0;
        const double h = top ? c.half_inv_M : 0.5 * inv_hi; // 1 / (2 sigma_{i+1})
        const double g = c.T * (r_hi - r_lo);
        const double m = c.m[i + 1];
        const double q = g * (2.0 * sig_lo + 2.0 * m + g) * (g + 2.0 * m) * (2.0 * sig_lo + g);
        const double pd = sqrt_pos(q) * h;
        w *= pd;
        if constexpr (KIN) {
            double ut, up;
            draw_angles_down<N>(rng, i, d.carry, phi_next, ut, up);
            double de = level_energy(m, sig_lo, g, sig_hi, h);
            double re = level_energy(sig_lo, m, g, sig_hi, h); // energy of {0..i}
            double dx, dy, dz;
            level_momentum(pd, ut, up, tab, dx, dy, dz);
            double rx = -dx, ry = -dy, rz = -dz;
            if (!top) {
                const double ex = px * inv_hi, ey = py * inv_hi, ez = pz * inv_hi;
                const double gamma = pe * inv_hi;
                const double inv_gp1 = sig_hi * recip(pe + sig_hi);
                boost<double>(de, dx, dy, dz, ex, ey, ez, gamma, inv_gp1);
                boost<double>(re, rx, ry, rz, ex, ey, ez, gamma, inv_gp1);
            }
            emit(i + 1, de, dx, dy, dz);
            if (i == 0) emit(0, re, rx, ry, rz);
            pe = re;
            px = rx;
            py = ry;
            pz = rz;
            // From six daughters keep each level's work together: without this
            // fence the scheduler hoists later levels' draws and square roots and
            // holds them live (N = 6..10: 2-4% slower without it; N = 3, 4: about
            // 0.5% faster without it).
            if constexpr (N >= 6) __builtin_amdgcn_sched_barrier(0);
        }
        sig_hi = sig_lo;
        inv_hi = inv_lo;
    }
    return w;
}

// One daughter from the parent's rest frame into the lab (moving parents).
__device__ __forceinline__ void boost_to_lab(double& e, double& x, double& y, double& z, const Frame& f) {
    boost<double>(e, x, y, z, f.eta[0], f.eta[1], f.eta[2], f.gamma, f.inv_gp1);
}

// The block's copy of the (cos, sin) table: filled once per block from the
// library's device table (block size >= kTrigSize), then read per lane.
__device__ __forceinline__ void load_trig(double2* lds, const double2* global) {
    if (threadIdx.x < kTrigSize) lds[threadIdx.x] = global[threadIdx.x];
    __syncthreads();
}

} // namespace hphsp
