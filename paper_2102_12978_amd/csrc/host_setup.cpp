// Host-side set-up in double precision: grid validation, periodic z fit,
// CPML coefficient tables, the antenna point set with its analytic Bessel
// amplitudes, and the temporal factor of the injected fields.
#include <cmath>
#include <complex>
#include <cstdio>
#include <string>
#include <vector>

#include "fdtd_internal.hpp"

namespace bfdtd {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC = 299792458.0;

double round_half_up(double x) { return std::floor(x + 0.5); }

// J_ν(x) for integer ν of either sign: J_{-ν} = (-1)^ν J_ν.
double bessel_j(int nu, double x) {
    int a = nu < 0 ? -nu : nu;
    double v = std::cyl_bessel_j(static_cast<double>(a), x);
    return (nu < 0 && (a & 1)) ? -v : v;
}

// J_ν(K r) e^{iνφ}
std::complex<double> bessel_term(int nu, double kr, double phi) {
    return bessel_j(nu, kr) * std::polar(1.0, nu * phi);
}

}  // namespace

std::string validate_grid(const fdtd_grid& g) {
    char buf[256];
    if (g.nx < 2 || g.ny < 2 || g.nz < 1) return "grid sizes must be nx, ny >= 2, nz >= 1";
    if ((long long)g.nx * g.ny * g.nz > (1LL << 34)) return "grid too large";
    if (!(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0)) return "cell sizes must be positive";
    if (!(g.courant > 0)) return "Courant number must be positive";
    double sx = g.courant, sy = g.courant * g.dx / g.dy, sz = g.courant * g.dx / g.dz;
    double cfl = std::sqrt(sx * sx + sy * sy + sz * sz);
    if (!(cfl < 1.0)) {
        std::snprintf(buf, sizeof buf, "Courant condition violated: S*sqrt(sum (dx/d)^2) = %.6f",
                      cfl);
        return buf;
    }
    if (g.bc_xy != FDTD_BC_CPML && g.bc_xy != FDTD_BC_PEC && g.bc_xy != FDTD_BC_PERIODIC)
        return "unknown bc_xy";
    if (g.bc_xy == FDTD_BC_CPML) {
        if (g.cpml_cells < 1 || 2 * g.cpml_cells > g.nx || 2 * g.cpml_cells > g.ny)
            return "cpml_cells must satisfy 1 <= cpml_cells <= min(nx, ny)/2";
        if (!(g.cpml_grade >= 0) || !(g.cpml_sigma_scale >= 0) || !(g.cpml_kappa_max >= 1) ||
            !(g.cpml_alpha_max >= 0))
            return "CPML parameters out of range";
    } else if (g.cpml_cells != 0) {
        return "cpml_cells must be 0 without a CPML boundary";
    }
    if (g.kernel < FDTD_KERNEL_AUTO || g.kernel > FDTD_KERNEL_FUSED) return "unknown kernel";
    return "";
}

void cpml_axis_tables(int n, int npml, double delta_ratio, const fdtd_grid& g, double dt,
                      std::vector<float>* tabs) {
    for (int t = 0; t < 6; ++t) tabs[t].assign(n, 0.0f);
    for (int i = 0; i < n; ++i) {
        tabs[T_EK][i] = 1.0f;
        tabs[T_HK][i] = 1.0f;
    }
    if (npml <= 0) return;
    const double smax = g.cpml_sigma_scale * 0.8 * (g.cpml_grade + 1.0) / delta_ratio;
    for (int half = 0; half < 2; ++half) {
        for (int i = 0; i < n; ++i) {
            double x = i + (half ? 0.5 : 0.0);
            double depth = std::fmax(std::fmax(npml - x, x - (n - npml)), 0.0);
            if (!(depth > 0)) continue;
            double rho = depth / npml;
            double pg = std::pow(rho, g.cpml_grade);
            double sigma = smax * pg;
            double kappa = 1.0 + (g.cpml_kappa_max - 1.0) * pg;
            double alpha = g.cpml_alpha_max * (1.0 - rho);
            double b = std::exp(-(sigma / kappa + alpha) * dt);
            double den = sigma * kappa + kappa * kappa * alpha;
            double c = den > 0 ? sigma * (b - 1.0) / den : 0.0;
            int o = half ? T_HB : T_EB;
            tabs[o][i] = (float)b;
            tabs[o + 1][i] = (float)c;
            tabs[o + 2][i] = (float)(1.0 / kappa);
        }
    }
}

void time_factor(const Antenna& a, double t, double* re, double* im) {
    double f = 1.0;
    if (a.ramp_kind == FDTD_RAMP_SIN2) {
        if (t < a.ramp_a) {
            double s = std::sin(0.5 * kPi * t / a.ramp_a);
            f = s * s;
        }
    } else if (a.ramp_kind == FDTD_RAMP_GAUSS) {
        double u = (t - a.ramp_b) / a.ramp_a;
        f = std::exp(-u * u);
    }
    double ph = -a.omega * (t - a.t0);
    *re = f * std::cos(ph);
    *im = f * std::sin(ph);
}

// Q = ∇×Π and R = ∇×Q of the potential J_m(K r) e^{imφ} e^{iβz} carried
// along x, y or z (pot 0, 1, 2), in the Cartesian forms printed in §3.1,
// without the common factor e^{iβz}.
void qr_fields(int pot, int m, double K, double beta, double k, double kr, double phi,
               std::complex<double> q[3], std::complex<double> r[3]) {
    const std::complex<double> I(0.0, 1.0);
    auto u = [&](int nu) { return bessel_term(nu, kr, phi); };
    const double kk = 0.5 * (k * k + beta * beta), k4 = 0.25 * K * K, bk = 0.5 * beta * K;
    if (pot == 0) {
        q[0] = 0.0;
        q[1] = I * beta * u(m);
        q[2] = (K / (2.0 * I)) * (u(m + 1) + u(m - 1));
        r[0] = kk * u(m) + k4 * (u(m + 2) + u(m - 2));
        r[1] = I * k4 * (u(m - 2) - u(m + 2));
        r[2] = I * bk * (u(m - 1) - u(m + 1));
    } else if (pot == 1) {
        q[0] = -I * beta * u(m);
        q[1] = 0.0;
        q[2] = -0.5 * K * (u(m + 1) - u(m - 1));
        r[0] = I * k4 * (u(m - 2) - u(m + 2));
        r[1] = kk * u(m) - k4 * (u(m + 2) + u(m - 2));
        r[2] = -bk * (u(m + 1) + u(m - 1));
    } else {
        q[0] = I * (0.5 * K) * (u(m + 1) + u(m - 1));
        q[1] = 0.5 * K * (u(m + 1) - u(m - 1));
        q[2] = 0.0;
        r[0] = -I * bk * (u(m + 1) - u(m - 1));
        r[1] = -bk * (u(m + 1) + u(m - 1));
        r[2] = K * K * u(m);
    }
}

std::string build_antenna(const fdtd_grid& g, int /*pitch*/, double ry, double rz,
                          const fdtd_injector& inj, Antenna* out) {
    Antenna a;
    if (!(inj.wavelength > 0)) return "wavelength must be positive";
    if (!(inj.theta > 0) || !(inj.theta < 0.5 * kPi)) return "theta must lie in (0, pi/2)";
    if (inj.order < 0 || inj.order > 64) return "order must lie in [0, 64]";
    if (!(inj.r_outer > 0) || !(inj.thickness > 0) || !(inj.thickness < inj.r_outer))
        return "antenna needs 0 < thickness < r_outer";
    if (!std::isfinite(inj.e0)) return "e0 must be finite";
    if (inj.ramp_kind == FDTD_RAMP_SIN2 && !(inj.ramp_a > 0)) return "sin2 ramp needs ramp_a > 0";
    if (inj.ramp_kind == FDTD_RAMP_GAUSS && !(inj.ramp_a > 0)) return "gauss ramp needs ramp_a > 0";
    if (inj.ramp_kind < FDTD_RAMP_SIN2 || inj.ramp_kind > FDTD_RAMP_CW) return "unknown ramp_kind";
    if (inj.n_sectors < 0) return "n_sectors must be >= 0";
    if (inj.polarization < FDTD_POL_X_TE || inj.polarization > FDTD_POL_Z_TM)
        return "polarization must be one of FDTD_POL_*";
    if (inj.n_sectors > 0 && (!inj.sector_amp || !inj.sector_phase))
        return "sector arrays required when n_sectors > 0";

    const double ns = inj.wavelength / g.dx;
    a.k = 2.0 * kPi / ns;
    a.kr = a.k * std::sin(inj.theta);
    a.beta = a.k * std::cos(inj.theta);
    a.omega = a.k;
    a.e0 = inj.e0;
    a.order = inj.order;
    a.theta = inj.theta;
    if (inj.flags & ~FDTD_INJ_ALLOW_Z_MISFIT) return "unknown injector flags";
    // the z phase must be periodic over the box, unless the caller accepts
    // the jump at the wrap
    double periods = a.beta * g.nz * rz / (2.0 * kPi);
    if (!(inj.flags & FDTD_INJ_ALLOW_Z_MISFIT) &&
        (std::fabs(periods - round_half_up(periods)) > 1e-6 || round_half_up(periods) < 1)) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "box length holds %.9f axial periods; use fdtd_fit_periodic_z", periods);
        return buf;
    }
    const double tunit = kC / g.dx;  // seconds -> Δx/c
    a.ramp_kind = inj.ramp_kind;
    a.ramp_a = inj.ramp_a * tunit;
    a.ramp_b = inj.ramp_b * tunit;
    a.t0 = inj.ramp_kind == FDTD_RAMP_GAUSS ? a.ramp_b : 0.0;
    a.ax = std::isnan(inj.axis_x) ? 0.5 * g.nx : inj.axis_x / g.dx;
    a.ay = std::isnan(inj.axis_y) ? 0.5 * g.ny * ry : inj.axis_y / g.dx;
    a.r_out = inj.r_outer / g.dx;
    a.r_in = (inj.r_outer - inj.thickness) / g.dx;
    a.n_sectors = inj.n_sectors;
    for (int s = 0; s < inj.n_sectors; ++s) {
        a.sec_amp.push_back(inj.sector_amp[s]);
        a.sec_phase.push_back(inj.sector_phase[s]);
    }

    static const double off[6][2] = {{0.5, 0.0}, {0.0, 0.5}, {0.0, 0.0},
                                     {0.0, 0.5}, {0.5, 0.0}, {0.5, 0.5}};
    const bool walls = g.bc_xy != FDTD_BC_PERIODIC;
    const int m = inj.order;
    const double k = a.k, K = a.kr, beta = a.beta, e0 = inj.e0;
    const int pot = inj.polarization % 3;              // potential along x, y, z
    const bool tm = inj.polarization >= FDTD_POL_X_TM;  // E from R (TM) or from Q (TE)
    a.polarization = inj.polarization;
    for (int j = 0; j < g.ny; ++j) {
        for (int i = 0; i < g.nx; ++i) {
            double bre[6] = {0}, bim[6] = {0};
            int mem[6] = {0}, sec[6] = {0};
            bool any = false;
            for (int c = 0; c < 6; ++c) {
                if (walls && (c == EY || c == EZ) && i == 0) continue;   // PEC tangential E
                if (walls && (c == EX || c == EZ) && j == 0) continue;
                double x = i + off[c][0] - a.ax;
                double y = (j + off[c][1]) * ry - a.ay;
                double r = std::hypot(x, y);
                if (!(r > a.r_in && r <= a.r_out)) continue;
                double phi = std::atan2(y, x);
                double kr = K * r;
                std::complex<double> q[3], rr[3];
                qr_fields(pot, m, K, beta, k, kr, phi, q, rr);
                const std::complex<double> I(0.0, 1.0);
                std::complex<double> v;
                if (c < 3)
                    v = tm ? (e0 / (k * k)) * rr[c] : (I * e0 / k) * q[c];
                else
                    v = tm ? (-I * e0 / k) * q[c - 3] : (e0 / (k * k)) * rr[c - 3];
                bre[c] = v.real();
                bim[c] = v.imag();
                mem[c] = 1;
                if (a.n_sectors > 0) {
                    double p = std::atan2(y, x);
                    if (p < 0) p += 2.0 * kPi;
                    int s = (int)(p * a.n_sectors / (2.0 * kPi));
                    sec[c] = s >= a.n_sectors ? a.n_sectors - 1 : s;
                }
                a.n_source[c] += 1;
                any = true;
            }
            if (!any) continue;
            a.slot_i.push_back(i);
            a.slot_j.push_back(j);
            for (int c = 0; c < 6; ++c) {
                a.base_re.push_back(bre[c]);
                a.base_im.push_back(bim[c]);
                a.member.push_back(mem[c]);
                a.sector.push_back(sec[c]);
            }
        }
    }
    *out = std::move(a);
    return "";
}

void weighted_amplitudes(const Antenna& a, std::vector<float>* out) {
    size_t ns = a.slot_i.size();
    out->assign(ns * 12, 0.0f);
    for (size_t s = 0; s < ns; ++s) {
        for (int c = 0; c < 6; ++c) {
            size_t q = s * 6 + c;
            std::complex<double> v(a.base_re[q], a.base_im[q]);
            if (a.n_sectors > 0 && a.member[q]) {
                int sec = a.sector[q];
                v *= std::polar(a.sec_amp[sec], a.sec_phase[sec]);
            }
            (*out)[q * 2] = (float)v.real();
            (*out)[q * 2 + 1] = (float)v.imag();
        }
    }
}

}  // namespace bfdtd
