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
    // the z phase must be periodic over the box
    double periods = a.beta * g.nz * rz / (2.0 * kPi);
    if (std::fabs(periods - round_half_up(periods)) > 1e-6 || round_half_up(periods) < 1) {
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
                std::complex<double> v;
                const std::complex<double> I(0.0, 1.0);
                switch (c) {
                    case EX: v = 0.0; break;
                    case EY: v = -(e0 * beta / k) * bessel_term(m, kr, phi); break;
                    case EZ:
                        v = (e0 * K / (2.0 * k)) *
                            (bessel_term(m + 1, kr, phi) + bessel_term(m - 1, kr, phi));
                        break;
                    case HX:
                        v = (e0 / (k * k)) *
                            (0.5 * (k * k + beta * beta) * bessel_term(m, kr, phi) +
                             0.25 * K * K * (bessel_term(m + 2, kr, phi) + bessel_term(m - 2, kr, phi)));
                        break;
                    case HY:
                        v = (e0 / (k * k)) * (0.25 * K * K * I) *
                            (bessel_term(m - 2, kr, phi) - bessel_term(m + 2, kr, phi));
                        break;
                    default:  // HZ
                        v = (e0 / (k * k)) * (0.5 * beta * K * I) *
                            (bessel_term(m - 1, kr, phi) - bessel_term(m + 1, kr, phi));
                        break;
                }
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
