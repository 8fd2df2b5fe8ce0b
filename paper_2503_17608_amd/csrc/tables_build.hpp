// Device construction of the physics tables (FP64) from the loaded materials
// and the production/tracking cut.  One thread per (material, node) evaluates
// the closed-form macroscopic cross sections; one thread per (material,
// species, grid interval) integrates 1/S with an 8-point Gauss-Legendre rule in
// ln T; one thread per (material, species) then accumulates the ranges.
#pragma once
#include "common.hpp"

namespace ems {

struct MatDev {
    double Z, A, rho, I_eV;
};

__device__ __forceinline__ double n_atoms(const MatDev& m) { return m.rho * kNA / m.A; }
__device__ __forceinline__ double x0_cm(const MatDev& m)
{
    // radiation length, PDG fit: 716.4 A / (Z (Z + 1) ln(287 / sqrt Z)) g/cm^2
    return 716.4 * m.A / (m.Z * (m.Z + 1.0) * log(287.0 / sqrt(m.Z))) / m.rho;
}

// Klein-Nishina total cross section per electron
__device__ double d_sigma_kn(double E)
{
    double k = E / kMe;
    double l = log(1.0 + 2.0 * k);
    double t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k);
    double t2 = l / (2.0 * k);
    double t3 = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
    return 2.0 * kPi * kRe * kRe * (t1 + t2 - t3);
}

// Born K-shell photoelectric cross section per atom, x 5/4 for all shells
__device__ double d_sigma_pe(double E, double Z)
{
    double sig_t = 8.0 * kPi * kRe * kRe / 3.0;
    double a2 = kAlpha * kAlpha;
    double z2 = Z * Z;
    return 1.25 * 4.0 * sqrt(2.0) * (a2 * a2) * (z2 * z2 * Z) * sig_t * pow(kMe / E, 3.5);
}

// complete-screening pair production, macroscopic
__device__ double d_sigma_pair(double E, double X0)
{
    if (E <= 2.0 * kMe) return 0.0;
    double a = kMe / E;
    double J = (1.0 - 2.0 * a) / 2.0 - (1.0 - 3.0 * a + 3.0 * a * a - 2.0 * a * a * a) / 3.0;
    return ((1.0 - 2.0 * a) - 4.0 / 3.0 * J) / X0;
}

__device__ double d_sigma_moller(double T, double Ec)
{
    if (T <= 2.0 * Ec) return 0.0;
    double g = (T + kMe) / kMe, b2 = 1.0 - 1.0 / (g * g), xc = Ec / T;
    double C1 = ((g - 1.0) / g) * ((g - 1.0) / g);
    double C2 = (2.0 * g - 1.0) / (g * g);
    double br = C1 * (0.5 - xc) + 1.0 / xc - 1.0 / (1.0 - xc) - C2 * log((1.0 - xc) / xc);
    return 2.0 * kPi * kRe * kRe / (b2 * (g - 1.0)) * br;
}

__device__ double d_sigma_bhabha(double T, double Ec)
{
    if (T <= Ec) return 0.0;
    double g = (T + kMe) / kMe, b2 = 1.0 - 1.0 / (g * g), xc = Ec / T;
    double y = 1.0 / (1.0 + g);
    double B1 = 2.0 - y * y;
    double B2 = (1.0 - 2.0 * y) * (3.0 + y * y);
    double B4 = (1.0 - 2.0 * y) * (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double B3 = B4 + (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double br = (1.0 / xc - 1.0) / b2 - B1 * log(1.0 / xc) + B2 * (1.0 - xc) - B3 * (1.0 - xc * xc) / 2.0 +
                B4 * (1.0 - xc * xc * xc) / 3.0;
    return 2.0 * kPi * kRe * kRe / (g - 1.0) * br;
}

__device__ double d_sigma_brems(double T, double Ec, double X0)
{
    if (T <= Ec) return 0.0;
    double E = T + kMe, yc = Ec / E, ym = T / E;
    return (4.0 / 3.0 * log(ym / yc) - 4.0 / 3.0 * (ym - yc) + (ym * ym - yc * yc) / 2.0) / X0;
}

// radiative loss to photons below min(Ec, T)
__device__ double d_srad(double T, double Ec, double X0)
{
    double E = T + kMe;
    double yr = fmin(Ec, T) / E;
    return E / X0 * (4.0 / 3.0 * yr - 2.0 / 3.0 * yr * yr + yr * yr * yr / 3.0);
}

// restricted collision stopping power (Berger-Seltzer) with the clamped
// high-energy density-effect correction
__device__ double d_scol(double T, double Ec, const MatDev& m, bool positron)
{
    double g = (T + kMe) / kMe, b2 = 1.0 - 1.0 / (g * g), tau = T / kMe;
    double Im = m.I_eV * 1.0e-6 / kMe;
    double F;
    if (positron) {
        double D = fmin(Ec, T) / kMe;
        double y = 1.0 / (g + 1.0);
        double D2 = D * D, D3 = D2 * D, D4 = D3 * D;
        F = log(tau * D) - b2 / tau *
                               (tau + 2.0 * D - 1.5 * D2 * y - (D - D3 / 3.0) * y * y -
                                (D2 / 2.0 - tau * D3 / 3.0 + D4 / 4.0) * y * y * y);
    } else {
        double D = fmin(Ec, T / 2.0) / kMe;
        F = -1.0 - b2 + log((tau - D) * D) + tau / (tau - D) +
            (D * D / 2.0 + (2.0 * tau + 1.0) * log(1.0 - D / tau)) / (g * g);
    }
    double bg = sqrt(b2) * g;
    double hwp = kPlasma * sqrt(m.rho * m.Z / m.A);
    double delta = fmax(0.0, 2.0 * log(hwp / m.I_eV) + 2.0 * log(bg) - 1.0);
    double L = log(2.0 * (tau + 2.0) / (Im * Im)) + F - delta;
    double n_el = m.Z * n_atoms(m);
    return 2.0 * kPi * kRe * kRe * kMe * n_el / b2 * L;
}

__device__ double d_stopping(double T, double Ec, const MatDev& m, bool positron)
{
    return d_scol(T, Ec, m, positron) + d_srad(T, Ec, x0_cm(m));
}

// radiation length of every material, for the multiple-scattering width
__global__ void k_material_x0(const MatDev* mats, int n_mat, double* x0)
{
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n_mat) x0[m] = x0_cm(mats[m]);
}

__global__ void k_build_xs(const MatDev* mats, int n_mat, double ecut, double ln_e0, double dlog, double* out)
{
    int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_mat * kNodes) return;
    int m = id / kNodes, i = id % kNodes;
    MatDev md = mats[m];
    double E = exp(ln_e0 + (double)i * dlog);
    double na = n_atoms(md), ne = md.Z * na, X0 = x0_cm(md);
    double* base = out + (size_t)m * kTabPerMat * kNodes;
    base[TB_COMPTON * kNodes + i] = ne * d_sigma_kn(E);
    base[TB_PHOTO * kNodes + i] = na * d_sigma_pe(E, md.Z);
    base[TB_PAIR * kNodes + i] = d_sigma_pair(E, X0);
    base[TB_MOLLER * kNodes + i] = ne * d_sigma_moller(E, ecut);
    base[TB_BHABHA * kNodes + i] = ne * d_sigma_bhabha(E, ecut);
    base[TB_BREMS * kNodes + i] = d_sigma_brems(E, ecut, X0);
}

// 8-point Gauss-Legendre nodes and weights on [-1, 1], ascending
__constant__ double c_gl_x[8] = {-0.9602898564975362, -0.7966664774136267, -0.525532409916329,
                                 -0.18343464249564978, 0.18343464249564978, 0.525532409916329,
                                 0.7966664774136267, 0.9602898564975362};
__constant__ double c_gl_w[8] = {0.10122853629037669, 0.22238103445337434, 0.31370664587788705,
                                 0.36268378337836177, 0.36268378337836177, 0.31370664587788705,
                                 0.22238103445337434, 0.10122853629037669};

// increments[m][species][i] = integral of dT/S over grid interval i
__global__ void k_range_increments(const MatDev* mats, int n_mat, double ecut, double ln_e0, double dlog,
                                   double* incr)
{
    int id = blockIdx.x * blockDim.x + threadIdx.x;
    int per = 2 * (kNodes - 1);
    if (id >= n_mat * per) return;
    int m = id / per, rem = id % per, sp = rem / (kNodes - 1), i = rem % (kNodes - 1);
    MatDev md = mats[m];
    double ua = ln_e0 + (double)i * dlog;
    double half = 0.5 * dlog;
    double mid = ua + half;
    double acc = 0.0;
    for (int k = 0; k < 8; ++k) {
        double t = exp(mid + half * c_gl_x[k]);
        acc += c_gl_w[k] * t / d_stopping(t, ecut, md, sp == 1);
    }
    incr[id] = half * acc;
}

__global__ void k_range_accumulate(const MatDev* mats, int n_mat, double ecut, double ln_e0, const double* incr,
                                   double* out)
{
    int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_mat * 2) return;
    int m = id / 2, sp = id % 2;
    MatDev md = mats[m];
    double E0 = exp(ln_e0);
    double* R = out + ((size_t)m * kTabPerMat + (sp ? TB_RANGE_EP : TB_RANGE_EM)) * kNodes;
    const double* in = incr + (size_t)id * (kNodes - 1);
    double r = E0 / d_stopping(E0, ecut, md, sp == 1);
    R[0] = r;
    for (int i = 0; i < kNodes - 1; ++i) {
        r = r + in[i];
        R[i + 1] = r;
    }
}

__global__ void k_tables_to_f32(const double* in, float* out, int n)
{
    int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n) out[id] = (float)in[id];
}

}  // namespace ems
