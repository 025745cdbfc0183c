// Host-side graph construction and validation (no HIP calls).
//
// QC block code (Eq. 2): J x L circulants of size p; block (j, l) with shift
// a >= 0 joins check j*p + s to variable l*p + (s + a) mod p.
// Convolutional code (Sec. II-C/II-D): check layer tau meets position
// tau - d through the syndrome-former component H_d(tau), a Jb x Lb array of
// circulants that depends on tau only through tau mod T.  Unwrapping a QC
// base with Lambda = gcd(J, L) gives T = Lambda, ms = Lambda - 1 and
// H_d(tau) = sub-block H_{tau mod T, (tau - d) mod T} of the base.
#include <algorithm>
#include <new>
#include <numeric>

#include "internal.h"

namespace {

constexpr int32_t kMaxP = 1 << 20;
constexpr int64_t kMaxEdges = int64_t(1) << 28;

bool shift_ok(int32_t a, int32_t p) { return a == -1 || (a >= 0 && a < p); }

ldpc_status fill_qc_desc(ldpc_graph* g) {
    ldpc::QCDesc& d = g->qc;
    d = ldpc::QCDesc{};
    d.J = g->J; d.L = g->L; d.p = g->p;
    int nb = 0;
    for (int j = 0; j < g->J; ++j) {
        d.rstart[j] = (uint16_t)nb;
        for (int l = 0; l < g->L; ++l) {
            int32_t a = g->shifts[j * g->L + l];
            if (a < 0) continue;
            if (nb >= LDPC_MAX_BLOCKS) return LDPC_EUNSUPPORTED;
            d.ecol[nb] = (uint8_t)l;
            d.eshift[nb] = a;
            ++nb;
        }
    }
    d.rstart[g->J] = (uint16_t)nb;
    d.nb = nb;
    int k = 0;
    for (int l = 0; l < g->L; ++l) {
        d.cstart[l] = (uint16_t)k;
        for (int b = 0; b < nb; ++b)
            if (d.ecol[b] == l) d.cedge[k++] = (uint16_t)b;   // b ascends with the base row
    }
    d.cstart[g->L] = (uint16_t)k;
    int dc = 0, dv = 0;
    for (int j = 0; j < g->J; ++j) dc = std::max(dc, d.rstart[j + 1] - d.rstart[j]);
    for (int l = 0; l < g->L; ++l) dv = std::max(dv, d.cstart[l + 1] - d.cstart[l]);
    if (dc > LDPC_MAX_ROW_WEIGHT || dv > LDPC_MAX_COL_WEIGHT) return LDPC_EUNSUPPORTED;
    int64_t E = (int64_t)nb * g->p;
    if (E > kMaxEdges || (int64_t)g->L * g->p > kMaxEdges) return LDPC_EUNSUPPORTED;
    d.n = g->L * g->p; d.m = g->J * g->p; d.E = (int32_t)E;
    d.dc_max = dc; d.dv_max = dv;
    g->n = d.n; g->m = d.m; g->E = d.E; g->dc_max = dc; g->dv_max = dv;
    g->rate = 1.0 - (double)g->J / (double)g->L;
    return LDPC_OK;
}

ldpc_status fill_conv_desc(ldpc_graph* g) {
    ldpc::ConvDesc& d = g->cv;
    d = ldpc::ConvDesc{};
    const int T = g->T, ms = g->ms, Jb = g->Jb, Lb = g->Lb, p = g->p;
    const int64_t entries = (int64_t)T * (ms + 1) * Jb * Lb;
    if (entries > LDPC_MAX_BLOCKS) return LDPC_EUNSUPPORTED;
    // the window kernels enumerate every syndrome-former slot of a row / column
    if ((ms + 1) * Lb > LDPC_MAX_ROW_WEIGHT || (ms + 1) * Jb > LDPC_MAX_COL_WEIGHT) return LDPC_EUNSUPPORTED;
    for (int64_t e = 0; e < entries; ++e) d.sf[e] = g->sf[e];
    d.T = T; d.ms = ms; d.Jb = Jb; d.Lb = Lb; d.p = p;
    d.c = Lb * p; d.cb = Jb * p;
    d.positions = g->positions; d.layers = g->layers;
    auto sf = [&](int i, int dd, int rr, int q) { return g->sf[((i * (ms + 1) + dd) * Jb + rr) * Lb + q]; };
    int dc = 0, dv = 0;
    for (int i = 0; i < T; ++i)
        for (int rr = 0; rr < Jb; ++rr) {
            int deg = 0;
            for (int dd = 0; dd <= ms; ++dd)
                for (int q = 0; q < Lb; ++q) deg += sf(i, dd, rr, q) >= 0;
            dc = std::max(dc, deg);
        }
    for (int jc = 0; jc < T; ++jc)
        for (int q = 0; q < Lb; ++q) {
            int deg = 0;
            for (int dd = 0; dd <= ms; ++dd)
                for (int rr = 0; rr < Jb; ++rr) deg += sf((jc + dd) % T, dd, rr, q) >= 0;
            dv = std::max(dv, deg);
        }
    if (dc > LDPC_MAX_ROW_WEIGHT || dv > LDPC_MAX_COL_WEIGHT) return LDPC_EUNSUPPORTED;
    int64_t E = 0;
    for (int64_t tau = 0; tau < g->layers; ++tau)
        for (int dd = 0; dd <= ms; ++dd) {
            int64_t t = tau - dd;
            if (t < 0 || t >= g->positions) continue;
            for (int rr = 0; rr < Jb; ++rr)
                for (int q = 0; q < Lb; ++q) E += (sf((int)(tau % T), dd, rr, q) >= 0) ? p : 0;
        }
    int64_t n = (int64_t)g->positions * Lb * p, m = (int64_t)g->layers * Jb * p;
    if (E > kMaxEdges || n > kMaxEdges || m > kMaxEdges) return LDPC_EUNSUPPORTED;
    d.dc_max = dc; d.dv_max = dv;
    g->n = (int32_t)n; g->m = (int32_t)m; g->E = (int32_t)E;
    g->dc_max = dc; g->dv_max = dv;
    g->rate = 1.0 - (double)Jb / (double)Lb;
    return LDPC_OK;
}

ldpc_status make_conv(ldpc_graph* g, int32_t positions, int32_t terminate) {
    g->kind = LDPC_GRAPH_CONV;
    g->positions = positions;
    g->terminate = terminate ? 1 : 0;
    g->layers = positions + (terminate ? g->ms : 0);
    return fill_conv_desc(g);
}

}  // namespace

extern "C" {

ldpc_status ldpc_graph_create_qc(const int32_t* shifts, int32_t J, int32_t L, int32_t p, ldpc_graph** out) {
    if (!out) return LDPC_EINVAL;
    *out = nullptr;
    if (!shifts || J <= 0 || L <= 0 || p <= 0) return LDPC_EINVAL;
    for (int64_t k = 0; k < (int64_t)J * L; ++k)
        if (!shift_ok(shifts[k], p)) return LDPC_EINVAL;
    if (J > LDPC_MAX_BASE_ROWS || L > LDPC_MAX_BASE_COLS || p > kMaxP) return LDPC_EUNSUPPORTED;
    ldpc_graph* g = new (std::nothrow) ldpc_graph();
    if (!g) return LDPC_ENOMEM;
    try {
        g->kind = LDPC_GRAPH_QC;
        g->J = J; g->L = L; g->p = p;
        g->shifts.assign(shifts, shifts + (size_t)J * L);
    } catch (...) {
        delete g;
        return LDPC_ENOMEM;
    }
    ldpc_status st = fill_qc_desc(g);
    if (st != LDPC_OK) { delete g; return st; }
    *out = g;
    return LDPC_OK;
}

ldpc_status ldpc_graph_create_ldpccc_from_qc(const int32_t* shifts, int32_t J, int32_t L, int32_t p,
                                             int32_t positions, int32_t terminate, ldpc_graph** out) {
    if (!out) return LDPC_EINVAL;
    *out = nullptr;
    if (!shifts || J <= 0 || L <= 0 || p <= 0 || positions <= 0) return LDPC_EINVAL;
    for (int64_t k = 0; k < (int64_t)J * L; ++k)
        if (!shift_ok(shifts[k], p)) return LDPC_EINVAL;
    if (J > LDPC_MAX_BASE_ROWS || L > LDPC_MAX_BASE_COLS || p > kMaxP) return LDPC_EUNSUPPORTED;
    const int32_t lam = std::gcd(J, L);
    ldpc_graph* g = new (std::nothrow) ldpc_graph();
    if (!g) return LDPC_ENOMEM;
    try {
        g->J = J; g->L = L; g->p = p;
        g->shifts.assign(shifts, shifts + (size_t)J * L);
        g->T = lam; g->ms = lam - 1; g->Jb = J / lam; g->Lb = L / lam;
        g->sf.assign((size_t)lam * lam * g->Jb * g->Lb, -1);
    } catch (...) {
        delete g;
        return LDPC_ENOMEM;
    }
    // H_d(tau) for layer class i = sub-block H_{i, (i - d) mod Lambda}
    for (int i = 0; i < lam; ++i)
        for (int dd = 0; dd < lam; ++dd) {
            int jc = ((i - dd) % lam + lam) % lam;
            for (int rr = 0; rr < g->Jb; ++rr)
                for (int q = 0; q < g->Lb; ++q)
                    g->sf[((i * lam + dd) * g->Jb + rr) * g->Lb + q] =
                        shifts[(i * g->Jb + rr) * L + jc * g->Lb + q];
        }
    ldpc_status st = make_conv(g, positions, terminate);
    if (st != LDPC_OK) { delete g; return st; }
    *out = g;
    return LDPC_OK;
}

ldpc_status ldpc_graph_create_ldpccc_sf(const int32_t* sf, int32_t T, int32_t ms, int32_t Jb, int32_t Lb,
                                        int32_t p, int32_t positions, int32_t terminate, ldpc_graph** out) {
    if (!out) return LDPC_EINVAL;
    *out = nullptr;
    if (!sf || T <= 0 || ms < 0 || Jb <= 0 || Lb <= 0 || p <= 0 || positions <= 0) return LDPC_EINVAL;
    const int64_t entries = (int64_t)T * (ms + 1) * Jb * Lb;
    if (entries > (int64_t)1 << 24) return LDPC_EUNSUPPORTED;
    for (int64_t k = 0; k < entries; ++k)
        if (!shift_ok(sf[k], p)) return LDPC_EINVAL;
    if (entries > LDPC_MAX_BLOCKS || p > kMaxP) return LDPC_EUNSUPPORTED;
    ldpc_graph* g = new (std::nothrow) ldpc_graph();
    if (!g) return LDPC_ENOMEM;
    try {
        g->p = p; g->T = T; g->ms = ms; g->Jb = Jb; g->Lb = Lb;
        g->sf.assign(sf, sf + entries);
    } catch (...) {
        delete g;
        return LDPC_ENOMEM;
    }
    ldpc_status st = make_conv(g, positions, terminate);
    if (st != LDPC_OK) { delete g; return st; }
    *out = g;
    return LDPC_OK;
}

ldpc_status ldpc_graph_get_info(const ldpc_graph* g, ldpc_graph_info* info) {
    if (!g || !info) return LDPC_EINVAL;
    ldpc_graph_info r{};
    r.kind = g->kind;
    r.n = g->n; r.m = g->m; r.E = g->E;
    r.dv_max = g->dv_max; r.dc_max = g->dc_max;
    r.J = g->J; r.L = g->L; r.p = g->p;
    if (g->kind == LDPC_GRAPH_CONV) {
        r.ms = g->ms; r.T = g->T; r.Jb = g->Jb; r.Lb = g->Lb;
        r.c = g->Lb * g->p; r.c_minus_b = g->Jb * g->p;
        r.positions = g->positions; r.layers = g->layers;
    }
    if (g->kind == LDPC_GRAPH_QC) {
        r.blocks = g->qc.nb;
    } else {
        for (int32_t v : g->sf) r.blocks += v >= 0 ? 1 : 0;
    }
    r.design_rate = g->rate;
    *info = r;
    return LDPC_OK;
}

void ldpc_graph_destroy(ldpc_graph* g) { delete g; }

const char* ldpc_status_str(ldpc_status s) {
    switch (s) {
        case LDPC_OK: return "ok";
        case LDPC_EINVAL: return "invalid argument";
        case LDPC_EWORKSPACE: return "workspace missing or too small";
        case LDPC_EHIP: return "HIP runtime error";
        case LDPC_EUNSUPPORTED: return "unsupported by this build";
        case LDPC_ENOMEM: return "host allocation failed";
    }
    return "unknown status";
}

}  // extern "C"
