// Host tables of the factorised D = 3, N = 4 coupling (k_couple4f): per
// (l1, l2) pair its slots (one per l3), per m3 the shared products
// a_{l1 m1} a_{l2 m2} and their coefficients for every slot (eq. Coupling-C
// with the CG of eq. CG-examples), and the wave tasks.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "npcf_internal.h"

namespace npcf {

// Factorised tables of the D = 3, N = 4 coupling (see FPair), and the wave
// tasks: jobs (pair, tile) paired heaviest with lightest so that every wave
// of a block carries about the same work.
void build_factorised(Tables &t, int L)
{
    t.fpairs.clear();
    t.fgroups.clear();
    t.fprods.clear();
    t.fcoef.clear();
    t.ftasks.clear();
    // every pair's l3 values must fit the slots (true for lmax <= 5); else the
    // term-by-term kernel is used
    for (int l1 = 0; l1 <= L; l1++)
        for (int l2 = 0; l2 <= L; l2++) {
            int n = 0;
            for (int lam = 0; lam < t.nlam; lam++)
                if (t.lam_lab[3 * lam] == l1 && t.lam_lab[3 * lam + 1] == l2) n++;
            if (n > kMaxSlots) return;
        }
    std::vector<double> cost;
    for (int l1 = 0; l1 <= L; l1++)
        for (int l2 = 0; l2 <= L; l2++) {
            FPair pr{};
            for (int lam = 0; lam < t.nlam; lam++) {
                const int *lb = &t.lam_lab[3 * lam];
                if (lb[0] == l1 && lb[1] == l2 && pr.nslot < kMaxSlots) {
                    pr.lam[pr.nslot] = lam;
                    pr.part[pr.nslot] = t.lam_part[lam];
                    pr.nslot++;
                }
            }
            if (pr.nslot == 0) continue;
            // slots by falling l3 (stable): the slots a group m3 reaches,
            // l3 >= m3, are then the first ones
            {
                int order[kMaxSlots];
                for (int k = 0; k < pr.nslot; k++) order[k] = k;
                std::stable_sort(order, order + pr.nslot, [&](int x, int y) {
                    return t.lam_lab[3 * pr.lam[x] + 2] > t.lam_lab[3 * pr.lam[y] + 2];
                });
                FPair sorted = pr;
                for (int k = 0; k < pr.nslot; k++) {
                    sorted.lam[k] = pr.lam[order[k]];
                    sorted.part[k] = pr.part[order[k]];
                }
                pr = sorted;
            }
            pr.grp_begin = (int)t.fgroups.size();
            double c_pair = 0.0;
            int l3max = 0;
            for (int k = 0; k < pr.nslot; k++) l3max = std::max(l3max, t.lam_lab[3 * pr.lam[k] + 2]);
            for (int m3 = 0; m3 <= l3max; m3++) {
                FGroup g{};
                g.prod_begin = (int)t.fprods.size();
                std::vector<int> m1s;
                for (int m1 = -l1; m1 <= l1; m1++) {
                    const int m2 = -m1 - m3;
                    if (std::abs(m2) > l2) continue;
                    FProd fp{};
                    fp.s1 = (int16_t)state_index(3, std::abs(m1), l1, 0);
                    fp.conj1 = m1 < 0;
                    fp.s2 = (int16_t)state_index(3, std::abs(m2), l2, 0);
                    fp.conj2 = m2 < 0;
                    t.fprods.push_back(fp);
                    m1s.push_back(m1);
                }
                g.prod_end = (int)t.fprods.size();
                const int np = g.prod_end - g.prod_begin;
                if (np == 0) continue;
                g.coef_begin = (int)t.fcoef.size();
                t.fcoef.resize(t.fcoef.size() + (size_t)kFCoefStride * np, 0.f);
                const double fold = (m3 > 0) ? 2.0 : 1.0;
                for (int k = 0; k < pr.nslot; k++) {
                    const int l3 = t.lam_lab[3 * pr.lam[k] + 2];
                    g.s3[k] = (int16_t)(l3 >= m3 ? state_index(3, m3, l3, 0) : 0);
                    if (l3 < m3) continue;
                    g.slot_mask |= 1 << k;
                    g.nact = k + 1;
                    for (int j = 0; j < np; j++) {
                        const int m1 = m1s[j], m2 = -m1 - m3;
                        // eq. Coupling-C: sum over M12 of <l1 m1, l2 m2 | l12 M12><l12 M12, l3 m3 | 0 0>, l12 = l3
                        double c = 0.0;
                        for (int M12 = -l3; M12 <= l3; M12++)
                            c += clebsch_gordan(l1, m1, l2, m2, l3, M12) * clebsch_gordan(l3, M12, l3, m3, 0, 0);
                        double sgn = 1.0;
                        if (m1 < 0 && (-m1) % 2) sgn = -sgn;
                        if (m2 < 0 && (-m2) % 2) sgn = -sgn;
                        t.fcoef[g.coef_begin + j * kFCoefStride + k] = (float)(fold * sgn * c);
                    }
                    c_pair += 2.0 * np + 8.0;  // FMAs into this slot's S and its MFMA slice
                }
                c_pair += 6.0 * np;            // products
                if (g.slot_mask != (1 << g.nact) - 1) {  // the kernel takes the active slots as a prefix
                    t.fpairs.clear();
                    t.fgroups.clear();
                    t.fprods.clear();
                    t.fcoef.clear();
                    return;
                }
                t.fgroups.push_back(g);
            }
            pr.grp_end = (int)t.fgroups.size();
            t.fpairs.push_back(pr);
            cost.push_back(c_pair);
        }
    // jobs (pair, tile) by falling cost.  One per wave: consecutive tasks share
    // a block (and its row steps), so a block holds jobs of similar cost.  Two
    // per wave: heaviest with lightest.
    std::vector<int> jobs;
    for (int pp = 0; pp < (int)t.fpairs.size(); pp++)
        for (int tile = 0; tile < t.mtiles; tile++) jobs.push_back(pp * t.mtiles + tile);
    std::stable_sort(jobs.begin(), jobs.end(),
                     [&](int x, int y) { return cost[x / t.mtiles] > cost[y / t.mtiles]; });
    if (kFJobsPerWave == 1) {
        for (int j : jobs) t.ftasks.push_back(make_int2(j, -1));
    } else {
        size_t lo = 0, hi = jobs.size();
        while (lo < hi) {
            int2 tk;
            tk.x = jobs[lo++];
            tk.y = (lo < hi) ? jobs[--hi] : -1;
            t.ftasks.push_back(tk);
        }
    }
}


}  // namespace npcf
