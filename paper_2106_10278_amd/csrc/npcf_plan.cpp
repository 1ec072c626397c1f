// Host planner of the NPCF library: validation, basis enumeration, coupling
// tables (eq. Coupling-C with the Clebsch-Gordan coefficients of eq.
// CG-examples), recurrence constants of the harmonics (Appendix A, eq.
// hypersph-def, in Gegenbauer form) and binning tables.  All in FP64 on the
// host; the device receives FP32/FP64 tables.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "npcf_internal.h"

namespace npcf {

namespace {

const int kLmaxD[5] = {0, 0, 16, 10, 6};

long double lfac(int n) { return std::lgamma((long double)n + 1.0L); }

// Normalisation of Gegenbauer polynomials: N(lambda, n)^2 * int_{-1}^{1}
// (1-x^2)^{lambda-1/2} [C^{(lambda)}_n(x)]^2 dx = 1, with the integral equal to
// pi 2^{1-2 lambda} Gamma(n+2 lambda) / (n! (n+lambda) Gamma(lambda)^2).

double dim_so(int D, int l)
{
    if (D == 2) return 1.0;
    if (D == 3) return 2.0 * l + 1.0;
    // D = 4: (l+1)^2 states of total angular momentum l
    return (double)(l + 1) * (l + 1);
}

}  // namespace

int state_index(int D, int l1, int l2, int l3)
{
    if (D == 2) return l1;
    if (D == 3) return l2 * (l2 + 1) / 2 + l1;
    return l3 * (l3 + 1) * (l3 + 2) / 6 + l2 * (l2 + 1) / 2 + l1;
}

double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3)
{
    // (j1 j2 j3; m1 m2 m3) = (-1)^{j1-j2-m3} <j1 m1, j2 m2 | j3, -m3> / sqrt(2 j3 + 1)
    const double cg = clebsch_gordan(j1, m1, j2, m2, j3, -m3);
    return (((j1 - j2 - m3) % 2) ? -cg : cg) / std::sqrt(2.0 * j3 + 1.0);
}

// <j1 m1, j2 m2 | J M> by Racah's closed form for the Clebsch-Gordan
// coefficient (sum over k with all factorial arguments non-negative).
double clebsch_gordan(int j1, int m1, int j2, int m2, int J, int M)
{
    if (M != m1 + m2) return 0.0;
    if (J < std::abs(j1 - j2) || J > j1 + j2) return 0.0;
    if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
    long double pre = 0.5L * (std::log(2.0L * J + 1.0L) + lfac(j1 + j2 - J) + lfac(j1 - j2 + J) + lfac(-j1 + j2 + J) -
                              lfac(j1 + j2 + J + 1) + lfac(j1 + m1) + lfac(j1 - m1) + lfac(j2 + m2) + lfac(j2 - m2) +
                              lfac(J + M) + lfac(J - M));
    long double sum = 0.0L;
    for (int k = 0; k <= j1 + j2 + J; k++) {
        int f1 = j1 + j2 - J - k, f2 = j1 - m1 - k, f3 = j2 + m2 - k, f4 = J - j2 + m1 + k, f5 = J - j1 - m2 + k;
        if (f1 < 0 || f2 < 0 || f3 < 0 || f4 < 0 || f5 < 0) continue;
        long double term = std::exp(pre - lfac(k) - lfac(f1) - lfac(f2) - lfac(f3) - lfac(f4) - lfac(f5));
        sum += (k % 2) ? -term : term;
    }
    return (double)sum;
}

npcf_status build_tables(const npcf_config &cfg, Tables &t, std::string &err)
{
    const int D = cfg.D, N = cfg.N, L = cfg.lmax, nb = cfg.nbins;
    if (D < 2 || D > 4 || N < 3 || N > 5) { err = "D must be 2..4 and N 3, 4 or 5"; return NPCF_E_UNSUPPORTED; }
    if (N == 4 && D == 4) { err = "N = 4 needs D <= 3 (no SO(4) coupling table)"; return NPCF_E_UNSUPPORTED; }
    if (N == 5 && D != 3) { err = "N = 5 needs D = 3"; return NPCF_E_UNSUPPORTED; }
    if (L < 0) { err = "lmax must be >= 0"; return NPCF_E_INVALID; }
    if (L > kLmaxD[D]) { err = "lmax above the supported maximum for this D"; return NPCF_E_UNSUPPORTED; }
    if (N == 5 && L > kLmax5) { err = "lmax above 5 for N = 5"; return NPCF_E_UNSUPPORTED; }
    if (nb < 1) { err = "nbins must be >= 1"; return NPCF_E_INVALID; }
    if (nb > kMaxBins) { err = "nbins above 16"; return NPCF_E_UNSUPPORTED; }
    if (!cfg.edges) { err = "edges is NULL"; return NPCF_E_INVALID; }
    for (int b = 0; b <= nb; b++)
        if (!std::isfinite(cfg.edges[b])) { err = "edges must be finite"; return NPCF_E_INVALID; }
    if (!(cfg.edges[0] > 0.0)) { err = "edges[0] must be > 0"; return NPCF_E_INVALID; }
    for (int b = 0; b < nb; b++)
        if (!(cfg.edges[b + 1] > cfg.edges[b])) { err = "edges must increase strictly"; return NPCF_E_INVALID; }
    if (cfg.geometry != NPCF_GEOMETRY_FLAT && cfg.geometry != NPCF_GEOMETRY_SPHERE &&
        cfg.geometry != NPCF_GEOMETRY_HYPERBOLIC) { err = "unknown geometry"; return NPCF_E_INVALID; }
    t.sphere = cfg.geometry != NPCF_GEOMETRY_FLAT;
    t.curv = cfg.geometry == NPCF_GEOMETRY_SPHERE ? 1 : (cfg.geometry == NPCF_GEOMETRY_HYPERBOLIC ? -1 : 0);
    if (t.curv < 0) {
        if ((D != 2 && D != 3) || N > 4 || cfg.basis != NPCF_BASIS_ISOTROPIC) { err = "hyperbolic space needs D = 2 or 3, N = 3 or 4 and the isotropic basis"; return NPCF_E_UNSUPPORTED; }
        if (L > kLmaxSphere) { err = "lmax above 5 in hyperbolic space"; return NPCF_E_UNSUPPORTED; }
        if (!(std::cosh(cfg.edges[0]) >= 1.0 + 1e-9)) { err = "hyperbolic edges[0] too small: cosh(edges[0]) must be at least 1 + 1e-9"; return NPCF_E_INVALID; }
        if (!(cfg.edges[nb] <= 20.0)) { err = "hyperbolic edges must not exceed 20"; return NPCF_E_INVALID; }
        if (!(cfg.box[0] > 0.0) || !std::isfinite(cfg.box[0])) { err = "hyperbolic space needs the region's volume V > 0 in box[0]"; return NPCF_E_INVALID; }
    } else if (t.sphere) {
        if ((D != 2 && D != 3) || N > 4 || cfg.basis != NPCF_BASIS_ISOTROPIC) { err = "the sphere needs D = 2 or 3, N = 3 or 4 and the isotropic basis"; return NPCF_E_UNSUPPORTED; }
        if (L > kLmaxSphere) { err = "lmax above 5 on the sphere"; return NPCF_E_UNSUPPORTED; }
        if (!(cfg.edges[nb] <= M_PI)) { err = "sphere edges must not exceed pi"; return NPCF_E_INVALID; }
        // bins are decided on cosines: the self pair (p.p = 1 up to rounding)
        // must lie outside the innermost edge
        if (!(std::cos(cfg.edges[0]) < 1.0 - 1e-12)) { err = "sphere edges[0] too small: cos(edges[0]) must be below 1 - 1e-12"; return NPCF_E_INVALID; }
    } else {
        for (int k = 0; k < D; k++) {
            if (!(cfg.box[k] > 0.0) || !std::isfinite(cfg.box[k])) { err = "box sides must be positive"; return NPCF_E_INVALID; }
            if (!(2.0 * cfg.edges[nb] < cfg.box[k])) { err = "need 2 * edges[nbins] < every box side"; return NPCF_E_INVALID; }
        }
    }
    if (cfg.btuple_mode != 0 && cfg.btuple_mode != 1) { err = "btuple_mode must be 0 or 1"; return NPCF_E_INVALID; }
    if (cfg.precision < 0 || cfg.precision > 3) { err = "unknown precision"; return NPCF_E_INVALID; }
    if (cfg.norm != 0 && cfg.norm != 1) { err = "unknown norm"; return NPCF_E_INVALID; }
    if (cfg.periodic != 0 && cfg.periodic != 1) { err = "periodic must be 0 or 1"; return NPCF_E_INVALID; }
    if (cfg.basis != NPCF_BASIS_ISOTROPIC && cfg.basis != NPCF_BASIS_LINE_OF_SIGHT) { err = "unknown basis"; return NPCF_E_INVALID; }
    const bool los = cfg.basis == NPCF_BASIS_LINE_OF_SIGHT;
    if (los && (D != 3 || N != 3)) { err = "the line-of-sight basis needs D = 3, N = 3"; return NPCF_E_UNSUPPORTED; }
    t.lab_w = N == 5 ? 5 : 3;
    t.bt_w = N == 5 ? 4 : 3;
    if (los && (cfg.Lmax < 0 || cfg.Lmax > 2 * L)) { err = "Lmax must be 0..2 lmax"; return NPCF_E_INVALID; }
    t.n3_terms = los;

    // ---- stored states (l1 >= 0 half) --------------------------------------
    t.nstate = stored_states(D, L);
    t.state_lab.assign(3 * t.nstate, 0);
    t.sfac.assign(t.nstate, 1.f);
    for (int l3 = 0; l3 <= (D == 4 ? L : 0); l3++)
        for (int l2 = 0; l2 <= (D == 2 ? 0 : (D == 3 ? L : l3)); l2++)
            for (int l1 = 0; l1 <= (D == 2 ? L : l2); l1++) {
                int s = state_index(D, l1, l2, l3);
                t.state_lab[3 * s] = l1;
                t.state_lab[3 * s + 1] = l2;
                t.state_lab[3 * s + 2] = l3;
                t.sfac[s] = (D >= 3 && l1 > 0) ? 2.f : 1.f;
            }

    // ---- Lambda labels ----------------------------------------------------------
    t.lam_lab.clear();
    if (los) {
        // (l1, l2, L): |l1 - l2| <= L <= min(l1 + l2, Lmax)
        for (int l1 = 0; l1 <= L; l1++)
            for (int l2 = 0; l2 <= L; l2++)
                for (int LL = std::abs(l1 - l2); LL <= std::min(l1 + l2, cfg.Lmax); LL++) {
                    t.lam_lab.push_back(l1);
                    t.lam_lab.push_back(l2);
                    t.lam_lab.push_back(LL);
                }
    } else if (N == 5) {
        // (l1, l2, l12, l3, l4): l12 by the triangle rule only, l4 <= lmax
        for (int l1 = 0; l1 <= L; l1++)
            for (int l2 = 0; l2 <= L; l2++)
                for (int l12 = std::abs(l1 - l2); l12 <= l1 + l2; l12++)
                    for (int l3 = 0; l3 <= L; l3++)
                        for (int l4 = std::abs(l12 - l3); l4 <= std::min(L, l12 + l3); l4++)
                            t.lam_lab.insert(t.lam_lab.end(), {l1, l2, l12, l3, l4});
    } else if (N == 3) {
        for (int l = 0; l <= L; l++) {
            t.lam_lab.push_back(l);
            t.lam_lab.push_back(D == 2 ? -l : 0);
            t.lam_lab.push_back(0);
        }
    } else if (D == 3) {
        for (int l1 = 0; l1 <= L; l1++)
            for (int l2 = 0; l2 <= L; l2++)
                for (int l3 = std::abs(l1 - l2); l3 <= std::min(L, l1 + l2); l3++) {
                    t.lam_lab.push_back(l1);
                    t.lam_lab.push_back(l2);
                    t.lam_lab.push_back(l3);
                }
    } else {
        for (int l1 = 0; l1 <= L; l1++)
            for (int l2 = -L; l2 <= L; l2++) {
                int l3 = -l1 - l2;
                if (std::abs(l3) > L) continue;
                t.lam_lab.push_back(l1);
                t.lam_lab.push_back(l2);
                t.lam_lab.push_back(l3);
            }
    }
    t.nlam = (int)t.lam_lab.size() / t.lab_w;
    t.nparts = (D == 2) ? 2 : 1;
    t.lam0 = 0;
    for (int i = 0; i < t.nlam; i++)
        if (std::all_of(&t.lam_lab[t.lab_w * i], &t.lam_lab[t.lab_w * (i + 1)], [](int v) { return v == 0; })) {
            t.lam0 = i;
            break;
        }

    // ---- radial tuples and GEMM row/column of each ------------------------------
    t.bt_lab.clear();
    t.row_pairs.clear();
    t.bt_row.clear();
    t.bt_col.clear();
    if (N == 5) {
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++)
                for (int b3 = 0; b3 < nb; b3++)
                    for (int b4 = 0; b4 < nb; b4++) {
                        if (cfg.btuple_mode == 0 && !(b1 < b2 && b2 < b3 && b3 < b4)) continue;
                        t.bt_lab.insert(t.bt_lab.end(), {b1, b2, b3, b4});
                    }
        t.row_pairs.push_back(make_int2(0, 0));
    } else if (N == 3) {
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++) {
                if (cfg.btuple_mode == 0 && !(b1 < b2)) continue;
                t.bt_lab.insert(t.bt_lab.end(), {b1, b2, 0});
                t.bt_row.push_back(b1);
                t.bt_col.push_back(b2);
            }
        t.mrows = nb;
        t.mtiles = 1;
    } else {
        std::vector<int> rowid(nb * nb, -1);
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++) {
                if (cfg.btuple_mode == 0 && !(b1 < b2 && b2 < nb - 1)) continue;
                rowid[b1 * nb + b2] = (int)t.row_pairs.size();
                t.row_pairs.push_back(make_int2(b1, b2));
            }
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++)
                for (int b3 = 0; b3 < nb; b3++) {
                    if (cfg.btuple_mode == 0 && !(b1 < b2 && b2 < b3)) continue;
                    t.bt_lab.insert(t.bt_lab.end(), {b1, b2, b3});
                    t.bt_row.push_back(rowid[b1 * nb + b2]);
                    t.bt_col.push_back(b3);
                }
        t.mrows = (int)t.row_pairs.size();
        t.mtiles = std::max(1, (t.mrows + 15) / 16);
        if (t.row_pairs.empty()) t.row_pairs.push_back(make_int2(0, 0));
    }
    t.nbt = (int)t.bt_lab.size() / t.bt_w;

    // ---- bins ------------------------------------------------------------------
    const double area = 2.0 * std::pow(M_PI, 0.5 * D) / std::tgamma(0.5 * D);
    t.e2.resize(nb + 1);
    t.vb.resize(nb);
    for (int b = 0; b <= nb; b++) t.e2[b] = cfg.edges[b] * cfg.edges[b];
    for (int b = 0; b < nb; b++) t.vb[b] = area * (std::pow(cfg.edges[b + 1], D) - std::pow(cfg.edges[b], D)) / D;
    double VD = 1.0;
    for (int k = 0; k < D; k++) VD *= cfg.box[k];
    if (t.curv < 0) {
        // bin volumes |S^{D-1}| int sinh^{D-1} r dr and the region's volume
        t.cedge.resize(nb + 1);
        for (int b = 0; b <= nb; b++) t.cedge[b] = -std::cosh(cfg.edges[b]);
        for (int b = 0; b < nb; b++) {
            if (D == 2) {
                t.vb[b] = 2.0 * M_PI * (std::cosh(cfg.edges[b + 1]) - std::cosh(cfg.edges[b]));
            } else {
                // 4 pi int sinh^2 = 2 pi ((sinh 2 e1 - sinh 2 e0) / 2 - d), with the
                // difference of sines as 2 cosh(e0 + e1) sinh d
                const double d = cfg.edges[b + 1] - cfg.edges[b];
                t.vb[b] = 2.0 * M_PI * (std::cosh(cfg.edges[b] + cfg.edges[b + 1]) * std::sinh(d) - d);
            }
        }
        VD = cfg.box[0];
    } else if (t.sphere) {
        // bin volumes |S^{D-1}| int sin^{D-1} r dr and the sphere's volume
        t.cedge.resize(nb + 1);
        for (int b = 0; b <= nb; b++) t.cedge[b] = std::cos(cfg.edges[b]);
        for (int b = 0; b < nb; b++) {
            if (D == 2) {
                t.vb[b] = 2.0 * M_PI * (t.cedge[b] - t.cedge[b + 1]);
            } else {
                // 4 pi int sin^2 = 2 pi (d - (sin 2 e1 - sin 2 e0) / 2), with the
                // difference of sines as 2 cos(e0 + e1) sin d
                const double d = cfg.edges[b + 1] - cfg.edges[b];
                t.vb[b] = 2.0 * M_PI * (d - std::cos(cfg.edges[b] + cfg.edges[b + 1]) * std::sin(d));
            }
        }
        VD = D == 2 ? 4.0 * M_PI : 2.0 * M_PI * M_PI;
    }
    t.bt_scale.resize(t.nbt);
    for (int i = 0; i < t.nbt; i++) {
        double p = VD;
        for (int k = 0; k < N - 1; k++) p *= t.vb[t.bt_lab[t.bt_w * i + k]];
        t.bt_scale[i] = 1.0 / p;
    }
    t.e2lo_f = (float)(t.e2[0] * (1.0 - 1e-5));
    t.e2hi_f = (float)(t.e2[nb] * (1.0 + 1e-5));
    const int nbucket = 1024;
    t.bucket_bin.resize(nbucket);
    t.bucket_lo = (float)t.e2[0];
    t.bucket_inv = (float)(nbucket / (t.e2[nb] - t.e2[0]));
    for (int k = 0; k < nbucket; k++) {
        double r2 = t.e2[0] + (t.e2[nb] - t.e2[0]) * k / nbucket;
        int b = 0;
        while (b + 1 < nb && r2 >= t.e2[b + 1]) b++;
        t.bucket_bin[k] = (uint8_t)b;
    }

    // ---- coupling groups and terms ----------------------------------------------------
    t.terms.clear();
    t.groups.clear();
    t.lam_group_begin.assign(1, 0);
    t.lam_part.assign(t.nlam, 0);
    if (N == 5) {
        for (int lam = 0; lam < t.nlam; lam++) {
            const int *lb = &t.lam_lab[5 * lam];
            t.lam_part[lam] = (lb[0] + lb[1] + lb[3] + lb[4]) % 2;
        }
        t.terms.push_back(CoupleTerm{});
        t.groups.push_back(CoupleGroup{});
        t.lam_group_begin.push_back(1);
        if (!build_c5(t, L, nb, cfg.btuple_mode)) { err = "too many outputs for N = 5"; return NPCF_E_UNSUPPORTED; }
        return NPCF_OK;
    }
    for (int lam = 0; lam < t.nlam; lam++) {
        const int *lb = &t.lam_lab[3 * lam];
        if (los) {
            // P^{0L}_{l1 l2} = (-1)^{l2-l1} sqrt(2L+1) sum_m (l1 l2 L; m -m 0) Y_{l1 m} Y_{l2,-m}
            // (section "Large-Scale Structure"); the prefactor times the 3j symbol is
            // the Clebsch-Gordan coefficient c_m = <l1 m, l2 -m | L 0>.  With
            // a_{l,-m} = (-1)^m conj(a_{l,m}) and c_{-m} = (-1)^{l1+l2+L} c_m, the terms
            // m and -m (m > 0) add to 2 (-1)^m c_m Re(a1 conj(a2)) (l1+l2+L even) or
            // i 2 (-1)^m c_m Im(a1 conj(a2)) (odd); m = 0 gives c_0 a1 a2 (real
            // states).  Terms: m = 0..min(l1, l2), legs (l1, m) and (l2, m).
            const int l1 = lb[0], l2 = lb[1], LL = lb[2];
            t.lam_part[lam] = (l1 + l2 + LL) % 2;
            CoupleGroup g{};
            g.term_begin = (int)t.terms.size();
            for (int m = 0; m <= std::min(l1, l2); m++) {
                const double c = clebsch_gordan(l1, m, l2, -m, LL, 0);
                if (c == 0.0) continue;
                CoupleTerm tm{};
                tm.s1 = (int16_t)state_index(3, m, l1, 0);
                tm.s2 = (int16_t)state_index(3, m, l2, 0);
                tm.coef = (float)((m > 0 ? 2.0 : 1.0) * ((m % 2) ? -1.0 : 1.0) * c);
                t.terms.push_back(tm);
            }
            g.term_end = (int)t.terms.size();
            t.groups.push_back(g);
        } else if (N == 3) {
            const int l = lb[0];
            CoupleGroup g{};
            if (D == 2) {
                g.s3 = l;
                g.nst = 1;
                g.scale3 = 1.f;
            } else {
                g.s3 = state_index(D, 0, D == 3 ? l : 0, l);
                g.nst = (D == 3) ? (l + 1) : (l + 1) * (l + 2) / 2;
                // C = (-1)^{l - l1} / sqrt(dim) for the pair ([l], (-l1, ...)); with
                // a_{(-l1)} = (-1)^{l1} conj(a_{l1}) the product is (-1)^l a conj(a) / sqrt(dim)
                g.scale3 = (float)(((l % 2) ? -1.0 : 1.0) / std::sqrt(dim_so(D, l)));
            }
            t.groups.push_back(g);
            t.lam_part[lam] = 0;
        } else if (D == 2) {
            const int l1 = lb[0], l2 = lb[1], l3 = lb[2];
            CoupleGroup g{};
            g.term_begin = (int)t.terms.size();
            CoupleTerm tm{};
            tm.s1 = (int16_t)l1;
            tm.conj1 = 0;
            tm.s2 = (int16_t)std::abs(l2);
            tm.conj2 = l2 < 0;
            tm.coef = 1.f;
            t.terms.push_back(tm);
            g.term_end = (int)t.terms.size();
            g.s3 = std::abs(l3);
            g.conj3 = l3 < 0;
            t.groups.push_back(g);
        } else {
            const int l1 = lb[0], l2 = lb[1], l3 = lb[2];
            t.lam_part[lam] = (l1 + l2 + l3) % 2;
            for (int m3 = 0; m3 <= l3; m3++) {
                CoupleGroup g{};
                g.term_begin = (int)t.terms.size();
                g.s3 = state_index(3, m3, l3, 0);
                g.conj3 = 0;
                const double fold = (m3 > 0) ? 2.0 : 1.0;
                for (int m1 = -l1; m1 <= l1; m1++) {
                    const int m2 = -m1 - m3;
                    if (std::abs(m2) > l2) continue;
                    // eq. Coupling-C: sum over M12 of <l1 m1, l2 m2 | l12 M12><l12 M12, l3 m3 | 0 0>, l12 = l3
                    double c = 0.0;
                    for (int M12 = -l3; M12 <= l3; M12++)
                        c += clebsch_gordan(l1, m1, l2, m2, l3, M12) * clebsch_gordan(l3, M12, l3, m3, 0, 0);
                    if (c == 0.0) continue;
                    CoupleTerm tm{};
                    double sgn = 1.0;
                    tm.s1 = (int16_t)state_index(3, std::abs(m1), l1, 0);
                    tm.conj1 = m1 < 0;
                    if (m1 < 0 && (-m1) % 2) sgn = -sgn;
                    tm.s2 = (int16_t)state_index(3, std::abs(m2), l2, 0);
                    tm.conj2 = m2 < 0;
                    if (m2 < 0 && (-m2) % 2) sgn = -sgn;
                    tm.coef = (float)(fold * sgn * c);
                    t.terms.push_back(tm);
                }
                g.term_end = (int)t.terms.size();
                if (g.term_end > g.term_begin) t.groups.push_back(g);
            }
        }
        t.lam_group_begin.push_back((int)t.groups.size());
    }
    if (t.terms.empty()) t.terms.push_back(CoupleTerm{});
    if (D == 3 && N == 4) build_factorised(t, L);   // npcf_plan4.cpp
    return NPCF_OK;
}

}  // namespace npcf
