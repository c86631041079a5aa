// Compile-time model of the derivative sums, shared by sph_forces and its
// adjoint: the smoothing kernel, the formulation, the laminar viscosity term
// and the density diffusion are template bits, so every combination is an
// instance of its own with no run-time branch in the pair loop (the
// template approach of section "Minimizing complexity" and listing
// l:ktemplate).  The instances of one smoothing kernel live in one
// translation unit, built with SPH_KERNEL_KIND set to that kernel.
#pragma once

#include <math.h>
#include <utility>

#include "sph_device.h"

namespace sph {

// model bits
constexpr int kViscBits = 3;          // laminar term: 0 none, 1 Morris, 2 Monaghan K form
constexpr int kMorris = 1, kMonaghanK = 2;
constexpr int kDiffusion = 4;         // Molteni-Colagrossi density diffusion between fluid particles
constexpr int kLandrini = 8;          // Landrini-Morris formulation (else the golden rule)
constexpr int kKernelShift = 4;       // smoothing kernel (SPH_KERNEL_*) in bits 4-5
constexpr int kModelLowBits = 15;     // everything but the kernel

constexpr int model_kernel(int m) { return (m >> kKernelShift) & 3; }
constexpr int model_visc(int m) { return m & kViscBits; }

// K of Monaghan's laminar form in 3D, d + 2: with the weight m_j/(rho_i rho_j)
// and the factor 2 mu_bar of the form, sum_j V_j (u_ij.x_ij) x_ij F_ij / r^2
// tends to (lap u + 2 grad div u) / (2 (d + 2)).
constexpr float kMonaghanKFactor = 5.0f;

// Model of a parameter set, -1 if one of its switches is unknown.
inline int model_of(const sph_params *p)
{
    if (p->visc_model < 0 || p->visc_model > 2) return -1;
    if (p->kernel < 0 || p->kernel > 3) return -1;
    if (p->formulation != 0 && p->formulation != 1) return -1;
    return p->visc_model | (p->delta != 0.0f ? kDiffusion : 0) | (p->formulation ? kLandrini : 0) |
           (p->kernel << kKernelShift);
}

// Coefficient c of F = c f(q) (host, double): the kernel's normalisation over h^5.
inline double kernel_coeff(int kind, double h)
{
    const double h5 = h * h * h * h * h;
    switch (kind) {
    case SPH_KERNEL_WENDLAND: return 105.0 / (128.0 * M_PI * h5);
    case SPH_KERNEL_CUBIC_SPLINE: return 1.0 / (M_PI * h5);
    case SPH_KERNEL_QUADRATIC: return 15.0 / (32.0 * M_PI * h5);
    case SPH_KERNEL_GAUSSIAN: {
        // W = C (exp(-q^2) - exp(-4)), F = -(2C/h^2) exp(-q^2)
        const double e4 = exp(-4.0);
        const double C = 1.0 / (4.0 * M_PI * h * h * h * (0.25 * sqrt(M_PI) * erf(2.0) - 11.0 / 3.0 * e4));
        return 2.0 * C / (h * h);
    }
    }
    return 0.0;
}

// Shape factors f(q) of F = c f(q):
//   Wendland (q - 2)^3;  cubic spline 9/4 q - 3 (q < 1), -3/4 (2 - q)^2 / q;
//   quadratic 1 - 2/q;  Gaussian -exp(-q^2).
// The cubic spline is evaluated without a select on q < 1 (one there makes the
// compiler split the unrolled pair loop and spill): with b = max(q, 1),
// f = 9/4 min(q - 1, 0) - 3/4 (2 - b)^2 / b takes the inner branch for q < 1
// (the second term is -3/4) and the outer one, to its own relative rounding,
// for q >= 1 (the first is 0), and f'(q) = 3/4 (2 - b)(2 + b) / b^2, which is
// 9/4 for q <= 1.  No term cancels and b >= 1, so F stays finite at r = 0.
// kernel_mF returns m_j F given mc = m_j c, r = sqrt(r2) (unused by the
// Gaussian, which needs only r2).
template <int KER>
__device__ __forceinline__ float kernel_mF(float mc, float r, float r2, float inv_h, float inv_h2)
{
    if constexpr (KER == SPH_KERNEL_WENDLAND) {
        const float qm2 = fmaf(r, inv_h, -2.0f);
        return (qm2 * qm2) * (qm2 * mc);
    } else if constexpr (KER == SPH_KERNEL_CUBIC_SPLINE) {
        const float q = r * inv_h;
        const float b = fmaxf(q, 1.0f), tb = 2.0f - b;
        return mc * fmaf(2.25f, fminf(q - 1.0f, 0.0f), -0.75f * tb * (tb * __builtin_amdgcn_rcpf(b)));
    } else if constexpr (KER == SPH_KERNEL_QUADRATIC) {
        const float q = r * inv_h;
        return mc * fmaf(-2.0f, __builtin_amdgcn_rcpf(q), 1.0f);
    } else {
        return -mc * __expf(-r2 * inv_h2);
    }
}

// F and F'(r)/r for the adjoint, c = kernel coefficient, inv_r = 1/r.
template <int KER>
__device__ __forceinline__ void kernel_F_dF(float c, float r, float r2, float inv_r, float inv_h, float inv_h2,
                                            float &F, float &Fp_r)
{
    if constexpr (KER == SPH_KERNEL_WENDLAND) {
        const float qm2 = fmaf(r, inv_h, -2.0f);
        const float cq = c * (qm2 * qm2);
        F = cq * qm2;
        Fp_r = cq * (3.0f * inv_h) * inv_r;
    } else if constexpr (KER == SPH_KERNEL_CUBIC_SPLINE) {
        const float q = r * inv_h;
        const float b = fmaxf(q, 1.0f), tb = 2.0f - b;
        const float ib = __builtin_amdgcn_rcpf(b);
        F = c * fmaf(2.25f, fminf(q - 1.0f, 0.0f), -0.75f * tb * (tb * ib));
        // dF/dr = (c/h) f'(q)
        Fp_r = c * inv_h * inv_r * (0.75f * tb * (2.0f + b) * ib * ib);
    } else if constexpr (KER == SPH_KERNEL_QUADRATIC) {
        const float q = r * inv_h;
        const float iq = __builtin_amdgcn_rcpf(q);
        F = c * fmaf(-2.0f, iq, 1.0f);
        Fp_r = 2.0f * c * iq * iq * inv_h * inv_r;
    } else {
        const float e = __expf(-r2 * inv_h2);
        F = -c * e;
        Fp_r = 2.0f * c * e * inv_h2;
    }
}

// Calls fn.template operator()<M>() for the model M of kernel KER whose low
// bits are `low`; false if `low` names no model.
template <int M, class Fn>
bool call_model(int low, Fn &fn)
{
    if constexpr (model_visc(M) == 3) {
        return false;
    } else {
        if (low != (M & kModelLowBits)) return false;
        fn.template operator()<M>();
        return true;
    }
}

template <int KER, class Fn, int... I>
bool with_model_impl(int low, Fn &fn, std::integer_sequence<int, I...>)
{
    return (call_model<I | (KER << kKernelShift)>(low, fn) || ...);
}

template <int KER, class Fn>
bool with_model(int low, Fn &&fn)
{
    return with_model_impl<KER>(low, fn, std::make_integer_sequence<int, kModelLowBits + 1>{});
}

}  // namespace sph
