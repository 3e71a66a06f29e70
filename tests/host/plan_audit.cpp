// Host-side audit of the workspace layout of the C ABI (test infrastructure,
// built with AddressSanitizer and UndefinedBehaviorSanitizer on the host pass
// only and run on the CPU).  It compiles in the library's own api.hip, so the
// planning and layout code under test is the code that ships, and drives the
// host-only part of the set-up path (box, neighbour parameters, DEM storage,
// workspace size, plan and layout) for the configurations the bench and the
// tests use, among them the 688,380-grain DEM avalanche with 16 contact slots.
// For each it checks that every array the kernels index lies inside the
// workspace, that arrays do not overlap, and that each array holds the
// extent its kernels address: per slot, per list entry, per caller-index row
// of the contact history (n x C), per cell and per particle workgroup.  No
// HIP call is made.  Exit status 0 when every check passes.
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "../../paper_1804_07598_amd/csrc/api.hip"

namespace {

int failures = 0;

void expect(bool ok, const char *what, const char *cfg) {
    if (!ok) {
        fprintf(stderr, "FAIL [%s] %s\n", cfg, what);
        failures++;
    }
}

struct Arr {
    const char *name;
    const void *p;
    size_t bytes;
};

void audit(const char *cfg, int nsys, const float *L, const int32_t *per, const int64_t *counts,
           int64_t n, float r_cut, float skin, int cap, int dem_cap) {
    fpm_ctx *c = nullptr;
    expect(fpm_create(&c, nullptr) == FPM_OK, "fpm_create", cfg);
    expect(fpm_set_systems(c, nsys, L, per, nsys > 1 ? counts : nullptr) == FPM_OK,
           "fpm_set_systems", cfg);
    expect(fpm_set_neighbor_params(c, r_cut, skin, cap) == FPM_OK, "fpm_set_neighbor_params",
           cfg);
    if (dem_cap) expect(fpm_set_dem(c, dem_cap) == FPM_OK, "fpm_set_dem", cfg);
    size_t bytes = 0;
    expect(fpm_workspace_size(c, n, &bytes) == FPM_OK, "fpm_workspace_size", cfg);
    std::vector<int64_t> cnt;
    expect(system_counts(c, n, cnt), "system counts", cfg);
    const Plan P = make_plan(c, cnt);
    // lay the workspace out at a fake base address (never dereferenced)
    char *base = reinterpret_cast<char *>(size_t(1) << 40);
    State s{};
    int32_t *pa = nullptr;
    const size_t used = layout(c, P, base, &s, &pa);
    expect(used == bytes, "layout size equals fpm_workspace_size", cfg);
    const int64_t ns = P.n_slots;
    int64_t ncall = 0;
    for (const SysDesc &d : P.desc) ncall += d.n;
    expect(ncall == n, "caller indices cover n", cfg);
    const size_t lst = (size_t)ns * cap4_for(cap) * 4;  // list entries (nbr_index range)
    std::vector<Arr> arrs = {
        {"pos0", s.pos[0], (ns + kPosSlack) * sizeof(float4)},
        {"pos1", s.pos[1], (ns + kPosSlack) * sizeof(float4)},
        {"vel0", s.vel[0], ns * sizeof(float4)},   {"vel1", s.vel[1], ns * sizeof(float4)},
        {"id0", s.id[0], ns * sizeof(int32_t)},    {"id1", s.id[1], ns * sizeof(int32_t)},
        {"frc", s.frc, ns * sizeof(float4)},       {"xbuild", s.xbuild, ns * sizeof(float4)},
        {"cid", s.cid, ns * sizeof(int32_t)},      {"rnk", s.rnk, ns * sizeof(int32_t)},
        {"tmp", s.tmp, ns * sizeof(int4)},
        {"cnt", s.cnt, (size_t)P.ncells_total * sizeof(int32_t)},
        {"off", s.off, (size_t)P.noff_total * sizeof(int32_t)},
        {"sub", s.sub, (size_t)P.ncells_total * 8 * sizeof(int32_t)},
        {"tsum", s.tsum, ((size_t)P.ncells_total / 4096 + 1) * sizeof(int32_t)},
        {"nbr", s.nbr, lst * sizeof(int32_t)},     {"nnb", s.nnb, ns * sizeof(uint32_t)},
        {"part", s.part, (size_t)P.nblk * kSlots * sizeof(double)},
        {"ring", s.ring, (size_t)P.nblk * kRingRows * 8 * sizeof(double)},
        {"aux", s.aux, ns * sizeof(float4)},       {"old0", s.old[0], ns * sizeof(float4)},
        {"old1", s.old[1], ns * sizeof(float4)},   {"ctl", s.ctl, sizeof(Ctl)},
        {"sctl", s.sctl, (size_t)nsys * sizeof(SysCtl)},
        {"sys", s.sys, (size_t)nsys * sizeof(SysDesc)},
        {"blk2sys", s.blk2sys, (size_t)P.nblk * sizeof(int32_t)},
        {"item2sys", s.item2sys, P.item2sys.size() * sizeof(int32_t)},
        {"blocks", pa, (P.pa_blocks.size() + P.grp_blocks.size() + P.ls_blocks.size()) *
                           sizeof(int32_t)},
    };
    if (dem_cap) {
        // history beside the list (one per list entry), caller-keyed rows of
        // the export (n x C partner ids and u_t), contact counts per grain
        arrs.push_back({"hl", s.hl, lst * sizeof(float4)});
        arrs.push_back({"hid", s.hid, (size_t)n * dem_cap * sizeof(int32_t)});
        arrs.push_back({"hu", s.hu, (size_t)n * dem_cap * sizeof(float4)});
        arrs.push_back({"ncon", s.ncon, (size_t)n * sizeof(int32_t)});
        // the clearing kernel's grid covers max(n C, list entries) threads
        expect((int64_t)std::max((size_t)n * dem_cap, lst) < (int64_t(1) << 31) * 256,
               "DEM clear grid fits the launch limit", cfg);
    }
    for (const Arr &a : arrs) {
        const char *p = static_cast<const char *>(a.p);
        expect(p != nullptr, a.name, cfg);
        expect(p >= base && p + a.bytes <= base + used, a.name, cfg);
        expect(((size_t)(p - base) % 256) == 0, a.name, cfg);
    }
    std::vector<Arr> sorted = arrs;
    std::sort(sorted.begin(), sorted.end(), [](const Arr &x, const Arr &y) { return x.p < y.p; });
    for (size_t k = 1; k < sorted.size(); k++)
        expect(static_cast<const char *>(sorted[k - 1].p) + sorted[k - 1].bytes <=
                   static_cast<const char *>(sorted[k].p),
               sorted[k].name, cfg);
    // tables: every workgroup and slot belongs to one system, slots cover n + padding
    int64_t slots = 0;
    for (size_t q = 0; q < P.desc.size(); q++) {
        const SysDesc &d = P.desc[q];
        expect(d.slot_base == slots && d.n_pad % kBlock == 0 && d.n_pad >= d.n + 1, "slots", cfg);
        expect(d.dummy == d.slot_base + d.n, "padding slot", cfg);
        slots += d.n_pad;
    }
    expect(slots == ns && (int64_t)P.nblk * kBlock == ns, "slot count", cfg);
    expect((int)P.blk2sys.size() == P.nblk, "workgroup table", cfg);
    // 32-bit byte offsets of the neighbour gathers
    expect(ns < (int64_t(1) << 28), "slots fit 32-bit byte offsets", cfg);
    fprintf(stderr, "ok [%s] n=%lld slots=%lld cells=%d workspace=%.1f MB arrays=%zu\n", cfg,
            (long long)n, (long long)ns, P.ncells_total, used / 1e6, arrs.size());
    expect(fpm_destroy(c) == FPM_OK, "fpm_destroy", cfg);
}

}  // namespace

int main() {
    const int32_t p111[3] = {1, 1, 1}, p010[3] = {0, 1, 0};
    {   // 1M-atom LJ liquid (rho 0.8442, default capacity)
        const float L[3] = {105.80793f, 105.80793f, 105.80793f};
        audit("lj1m", 1, L, p111, nullptr, 1000000, 2.5f, 0.3f, 176, 0);
    }
    {   // the DEM avalanche of the bench: 149 x 105 x 44 grains, R = 0.06
        const float L[3] = {8.4f * 4.2f, 3.0f * 4.2f, 3.18f * 4.2f};
        audit("dem688k", 1, L, p010, nullptr, 688380, 0.12f, 0.006f, 32, 16);
        audit("dem688k-C64", 1, L, p010, nullptr, 688380, 0.12f, 0.006f, 64, 64);
    }
    {   // a batch of uneven systems
        std::vector<float> L;
        std::vector<int32_t> per;
        std::vector<int64_t> cnt;
        int64_t n = 0;
        for (int s = 0; s < 64; s++) {
            const int64_t k = 256 + (s * 7919) % 7937;
            const float side = (float)cbrt((double)k / 0.75);
            for (int a = 0; a < 3; a++) L.push_back(side), per.push_back(1);
            cnt.push_back(k);
            n += k;
        }
        audit("batch64", 64, L.data(), per.data(), cnt.data(), n, 2.5f, 0.3f, 160, 0);
    }
    {   // the SPH column (non-periodic z)
        const int32_t pz[3] = {1, 1, 0};
        const float L[3] = {1.28f, 1.28f, 1.6f};
        audit("sph2m", 1, L, pz, nullptr, 2146304, 0.026f, 0.0013f, 176, 0);
    }
    if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
    return failures ? 1 : 0;
}
