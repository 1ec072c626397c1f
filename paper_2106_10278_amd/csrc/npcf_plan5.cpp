// Host tables of the isotropic 5PCF coupling (D = 3, N = 5; section
// "Hydrodynamic Turbulence"): see C5Job.  FP64 on the host, FP32 terms on the
// device.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "npcf_internal.h"

namespace npcf {

// Isotropic 5PCF tables (see C5Job): per l12 the S labels (l1, l2) and T
// labels (l3, l4) that couple to it, their per-M term lists, the jobs, and the
// accumulator index and sign of every output (Lambda, b-tuple).
bool build_c5(Tables &t, int L, int nb, int mode)
{
    const int L12 = 2 * L;
    std::vector<std::vector<int2>> pl(L12 + 1);
    for (int l12 = 0; l12 <= L12; l12++)
        for (int la = 0; la <= L; la++)
            for (int lb = 0; lb <= L; lb++)
                if (std::abs(la - lb) <= l12 && l12 <= la + lb) pl[l12].push_back(make_int2(la, lb));
    // a leg a_{l m} from the stored m >= 0 half: a_{l,-m} = (-1)^m conj(a_{l m})
    auto push_term = [&](int ma, int la, int mb, int lb, double c) {
        CoupleTerm tm{};
        double sg = 1.0;
        tm.s1 = (int16_t)state_index(3, std::abs(ma), la, 0);
        tm.conj1 = ma < 0;
        if (ma < 0 && (-ma) % 2) sg = -sg;
        tm.s2 = (int16_t)state_index(3, std::abs(mb), lb, 0);
        tm.conj2 = mb < 0;
        if (mb < 0 && (-mb) % 2) sg = -sg;
        tm.coef = (float)(sg * c);
        t.c5terms.push_back(tm);
    };
    std::vector<int> s_first(L12 + 1), t_first(L12 + 1);
    for (int l12 = 0; l12 <= L12; l12++)
        for (int side = 0; side < 2; side++) {
            (side == 0 ? s_first : t_first)[l12] = (int)t.c5labels.size();
            for (const int2 pr : pl[l12]) {
                const int la = pr.x, lb = pr.y;
                const double par = ((la + lb) % 2) ? -1.0 : 1.0;
                C5Label lab{};
                lab.mt = (int)t.c5mterm.size();
                lab.rot = (la + lb) % 2;
                for (int M = 0; M <= l12; M++) {
                    t.c5mterm.push_back((int)t.c5terms.size());
                    if (side == 0) {
                        // S_M: the first 3-j of the section's 5PCF form with m12 = M, times
                        // (-1)^{l1+l2} sqrt(2 l12 + 1) (-1)^{l12-M} and the +-M fold (2 for M > 0)
                        const double h = par * std::sqrt(2.0 * l12 + 1.0) * (((l12 - M) % 2) ? -1.0 : 1.0) * (M > 0 ? 2.0 : 1.0);
                        for (int m1 = -la; m1 <= la; m1++) {
                            const int m2 = M - m1;
                            if (std::abs(m2) > lb) continue;
                            const double c = wigner3j(la, lb, l12, m1, m2, -M);
                            if (c != 0.0) push_term(m1, la, m2, lb, h * c);
                        }
                    } else {
                        // T_M: the second 3-j with m12 = M, times (-1)^{l3+l4}
                        for (int m3 = -la; m3 <= la; m3++) {
                            const int m4 = -M - m3;
                            if (std::abs(m4) > lb) continue;
                            const double c = wigner3j(l12, la, lb, M, m3, m4);
                            if (c != 0.0) push_term(m3, la, m4, lb, par * c);
                        }
                    }
                }
                t.c5mterm.push_back((int)t.c5terms.size());
                t.c5labels.push_back(lab);
            }
        }
    // radial pairs (b3, b4) of each beta, and the jobs of each (l12, beta)
    std::vector<int> pair_begin(nb), npair(nb), pidx(nb * nb * nb, -1);
    for (int beta = 0; beta < nb; beta++) {
        pair_begin[beta] = (int)t.c5pairs.size();
        for (int b3 = 0; b3 < nb; b3++)
            for (int b4 = 0; b4 < nb; b4++) {
                if (mode == 0 && !(beta < b3 && b3 < b4)) continue;
                pidx[(beta * nb + b3) * nb + b4] = (int)t.c5pairs.size() - pair_begin[beta];
                t.c5pairs.push_back(make_int2(b3, b4));
            }
        npair[beta] = (int)t.c5pairs.size() - pair_begin[beta];
    }
    if (t.c5pairs.empty()) t.c5pairs.push_back(make_int2(0, 0));
    std::vector<int> first_job((L12 + 1) * nb, -1), spg_of((L12 + 1) * nb, 1), ncg_of((L12 + 1) * nb, 1);
    t.c5tiles = 0;
    for (int l12 = 0; l12 <= L12; l12++)
        for (int beta = 0; beta < nb; beta++) {
            const int nb1 = mode == 0 ? beta : nb;
            const int ns_all = (int)pl[l12].size();
            if (nb1 == 0 || npair[beta] == 0 || ns_all == 0) continue;
            const int spg = std::max(1, kC5Rows / nb1);
            const int ncol_all = ns_all * npair[beta];
            const int ncg = (ncol_all + kC5Cols - 1) / kC5Cols;
            first_job[l12 * nb + beta] = (int)t.c5jobs.size();
            spg_of[l12 * nb + beta] = spg;
            ncg_of[l12 * nb + beta] = ncg;
            for (int s0 = 0; s0 < ns_all; s0 += spg)
                for (int cg = 0; cg < ncg; cg++) {
                    C5Job j{};
                    j.l12 = l12;
                    j.beta = beta;
                    j.nb1 = nb1;
                    j.s_begin = s_first[l12] + s0;
                    j.ns = std::min(spg, ns_all - s0);
                    j.t_begin = t_first[l12];
                    j.col_begin = cg * kC5Cols;
                    j.ncol = std::min(kC5Cols, ncol_all - j.col_begin);
                    j.pair_begin = pair_begin[beta];
                    j.npair = npair[beta];
                    j.nrt = (j.ns * nb1 + 15) / 16;
                    j.tile_begin = t.c5tiles;
                    t.c5tiles += j.nrt * 4;
                    t.c5jobs.push_back(j);
                }
        }
    if ((int64_t)t.c5tiles * 256 > (int64_t)INT32_MAX || (int64_t)t.nlam * t.nbt > (1LL << 28)) return false;
    // device form of the terms, and the LDS a job's tables take: per label
    // l12 + 2 range entries and a phase flag, 8 bytes per term
    t.c5packed.clear();
    for (const CoupleTerm &tm : t.c5terms) {
        uint2 v;
        v.x = (uint32_t)(uint16_t)tm.s1 | ((uint32_t)(uint16_t)tm.s2 << 8) | ((uint32_t)(tm.conj1 != 0) << 16) |
              ((uint32_t)(tm.conj2 != 0) << 17);
        std::memcpy(&v.y, &tm.coef, 4);
        t.c5packed.push_back(v);
    }
    t.c5_lds_extra = 0;
    for (const C5Job &j : t.c5jobs) {
        const int nmt = j.l12 + 2;
        const int t0 = j.col_begin / j.npair, t1 = (j.col_begin + j.ncol - 1) / j.npair;
        const int ntl = t1 - t0 + 1;
        const C5Label &sf = t.c5labels[j.s_begin], &tf = t.c5labels[j.t_begin + t0];
        const int sterms = t.c5mterm[sf.mt + j.ns * nmt - 1] - t.c5mterm[sf.mt];
        const int tterms = t.c5mterm[tf.mt + ntl * nmt - 1] - t.c5mterm[tf.mt];
        const int bytes = 4 * (((j.ns + ntl) * (nmt + 1) + kC5Rows + 1) & ~1) + 8 * (sterms + tterms);
        t.c5_lds_extra = std::max(t.c5_lds_extra, (bytes + 15) / 16 * 16);
    }
    // accumulator index and sign of every output
    t.c5sign.assign(t.nlam, 1.0);
    t.c5idx.assign((size_t)t.nlam * t.nbt, 0);
    for (int lam = 0; lam < t.nlam; lam++) {
        const int *lb = &t.lam_lab[5 * lam];
        const int l12 = lb[2];
        int s = -1, tt = -1;
        for (int k = 0; k < (int)pl[l12].size(); k++) {
            if (pl[l12][k].x == lb[0] && pl[l12][k].y == lb[1]) s = k;
            if (pl[l12][k].x == lb[3] && pl[l12][k].y == lb[4]) tt = k;
        }
        // Re(S~ T~) is -Re(S T) when both phases are -i (even parity, odd l1 + l2)
        if (((lb[0] + lb[1]) % 2) && ((lb[3] + lb[4]) % 2)) t.c5sign[lam] = -1.0;
        for (int q = 0; q < t.nbt; q++) {
            const int *B = &t.bt_lab[4 * q];
            const int beta = B[1], key = l12 * nb + beta;
            const int nb1 = mode == 0 ? beta : nb;
            const int col = tt * npair[beta] + pidx[(beta * nb + B[2]) * nb + B[3]];
            const int sg = s / spg_of[key], cg = col / kC5Cols;
            const C5Job &j = t.c5jobs[first_job[key] + sg * ncg_of[key] + cg];
            const int row = (s - (j.s_begin - s_first[l12])) * nb1 + B[0];
            const int cl = col - j.col_begin;
            t.c5idx[(size_t)lam * t.nbt + q] = (j.tile_begin + (row / 16) * 4 + cl / 16) * 256 + (row % 16) * 16 + cl % 16;
        }
    }
    return true;
}

}  // namespace npcf
