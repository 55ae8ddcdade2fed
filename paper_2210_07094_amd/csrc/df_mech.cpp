// Mechanism loading: "dfmech 1" parser, device-table packing, handle lifetime,
// error reporting and option helpers of the C ABI.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "df_internal.h"

namespace df {

static thread_local std::string g_last_error;

df_status fail(df_status code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

void clear_error() { g_last_error.clear(); }

namespace {

// whitespace tokenizer that drops '#' comments to end of line
class Tokens {
   public:
    explicit Tokens(std::istream &in) {
        std::string line;
        while (std::getline(in, line)) {
            auto h = line.find('#');
            if (h != std::string::npos) line.resize(h);
            std::istringstream ls(line);
            std::string t;
            while (ls >> t) toks_.push_back(t);
        }
    }
    bool next(std::string &t) {
        if (pos_ >= toks_.size()) return false;
        t = toks_[pos_++];
        return true;
    }
    bool key(const char *k) {
        std::string t;
        return next(t) && t == k;
    }
    template <class T>
    bool num(T &v) {
        std::string t;
        if (!next(t)) return false;
        char *end = nullptr;
        if constexpr (std::is_integral_v<T>) {
            long x = std::strtol(t.c_str(), &end, 10);
            v = static_cast<T>(x);
        } else {
            v = std::strtod(t.c_str(), &end);
        }
        return end && *end == '\0';
    }
    template <class T>
    bool nums(std::vector<T> &v, size_t n) {
        v.resize(n);
        for (size_t i = 0; i < n; ++i)
            if (!num(v[i])) return false;
        return true;
    }

   private:
    std::vector<std::string> toks_;
    size_t pos_ = 0;
};

}  // namespace

df_status parse_mech_file(const char *path, HostMech &m) {
    std::ifstream f(path);
    if (!f) return fail(DF_E_IO, std::string("cannot open mechanism file ") + path);
    Tokens t(f);
    int ver = 0;
    std::string s;
    auto bad = [&](const char *what) { return fail(DF_E_FORMAT, std::string(path) + ": malformed section '" + what + "'"); };
    if (!t.key("dfmech") || !t.num(ver) || ver != 1) return bad("dfmech");
    if (!t.key("name") || !t.next(m.name)) return bad("name");
    if (!t.key("seed") || !t.num(m.seed)) return bad("seed");
    if (!t.key("n_elements") || !t.num(m.E) || m.E < 1) return bad("n_elements");
    if (!t.key("n_species") || !t.num(m.K) || m.K < 1) return bad("n_species");
    if (!t.key("n_reactions") || !t.num(m.M) || m.M < 0) return bad("n_reactions");
    const size_t E = m.E, K = m.K, M = m.M;
    if (!t.key("elements")) return bad("elements");
    for (size_t i = 0; i < E; ++i)
        if (!t.next(s)) return bad("elements");
    std::vector<double> emass;
    if (!t.key("element_mass") || !t.nums(emass, E)) return bad("element_mass");
    if (!t.key("species")) return bad("species");
    for (size_t i = 0; i < K; ++i)
        if (!t.next(s)) return bad("species");
    if (!t.key("molar_mass") || !t.nums(m.W, K)) return bad("molar_mass");
    for (auto &w : m.W) {
        if (!(w > 0)) return bad("molar_mass");
        w *= 1e-3;  // g/mol -> kg/mol
    }
    if (!t.key("composition") || !t.nums(m.comp, K * E)) return bad("composition");
    if (!t.key("nasa7") || !t.nums(m.nasa, K * 7)) return bad("nasa7");
    if (!t.key("reaction_type") || !t.nums(m.type, M)) return bad("reaction_type");
    if (!t.key("nu_reac") || !t.nums(m.nu_r, M * K)) return bad("nu_reac");
    if (!t.key("nu_prod") || !t.nums(m.nu_p, M * K)) return bad("nu_prod");
    if (!t.key("arrhenius") || !t.nums(m.arr, M * 3)) return bad("arrhenius");
    if (!t.key("efficiency") || !t.nums(m.eff, M * K)) return bad("efficiency");
    if (!t.key("falloff_low") || !t.nums(m.low, M * 3)) return bad("falloff_low");
    if (!t.key("troe") || !t.nums(m.troe, M * 4)) return bad("troe");
    if (!t.key("end")) return bad("end");
    for (size_t j = 0; j < M; ++j) {
        if (m.type[j] < 0 || m.type[j] > 2) return bad("reaction_type");
        if (!(m.arr[3 * j] > 0)) return bad("arrhenius");
        if (m.type[j] == 2 && !(m.low[3 * j] > 0)) return bad("falloff_low");
        int nr = 0, np = 0;
        for (size_t k = 0; k < K; ++k) {
            if (m.nu_r[j * K + k] < 0 || m.nu_p[j * K + k] < 0) return bad("nu");
            nr += m.nu_r[j * K + k];
            np += m.nu_p[j * K + k];
        }
        if (nr < 1 || np < 1) return bad("nu");
        if (nr > kSlots || np > kSlots)
            return fail(DF_E_UNSUPPORTED, std::string(path) + ": reaction with more than 3 molecules on a side");
    }
    return DF_OK;
}

// Order in which the reactions are stored on the device.  The cooperative kernel
// evaluates stored reaction j on lane j % 16, so the order spreads the costly
// reactions (Troe falloff: seven transcendentals; third body: a K-term sum) over
// the lanes: longest-processing-time assignment of reactions, in decreasing cost,
// to the lane with the least work that still has a free slot.  Results do not
// depend on the order beyond the summation order of production rates.
static std::vector<int> lane_balanced_order(const HostMech &m, int lanes = 16) {
    const int M = m.M;
    std::vector<int> slots(lanes, 0);
    for (int j = 0; j < M; ++j) ++slots[j % lanes];
    auto cost = [&](int j) { return m.type[j] == 2 ? 8.0 : (m.type[j] == 1 ? 1.5 : 1.0); };
    std::vector<int> byc(M);
    for (int j = 0; j < M; ++j) byc[j] = j;
    std::stable_sort(byc.begin(), byc.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<double> load(lanes, 0.0);
    std::vector<std::vector<int>> assigned(lanes);
    for (int j : byc) {
        int best = -1;
        for (int l = 0; l < lanes; ++l)
            if (int(assigned[l].size()) < slots[l] && (best < 0 || load[l] < load[best])) best = l;
        assigned[best].push_back(j);
        load[best] += cost(j);
    }
    std::vector<int> order(M);
    for (int l = 0; l < lanes; ++l)
        for (size_t q = 0; q < assigned[l].size(); ++q) order[l + q * lanes] = assigned[l][q];
    return order;
}

// Pack the host mechanism into the device table layout described in df_internal.h.
static void pack_tables(const HostMech &m, std::vector<double> &sp, std::vector<int> &rx, std::vector<double> &rk,
                        std::vector<double> &eff, std::vector<int> &nu, std::vector<int> &spl, int &lmax) {
    const int K = m.K, M = m.M;
    const std::vector<int> order = lane_balanced_order(m);
    sp.assign(size_t(K) * kSpTab, 0.0);
    for (int k = 0; k < K; ++k) {
        const double *a = &m.nasa[7 * k];
        double *r = &sp[size_t(k) * kSpTab];
        r[0] = m.W[k];
        r[1] = 1.0 / m.W[k];
        for (int i = 0; i < 7; ++i) r[2 + i] = a[i];
        r[9] = a[1] / 2;
        r[10] = a[2] / 3;
        r[11] = a[3] / 4;
        r[12] = a[4] / 5;
        r[13] = a[2] / 2;
        r[14] = a[3] / 3;
        r[15] = a[4] / 4;
        r[16] = 2 * a[2];
        r[17] = 3 * a[3];
        r[18] = 4 * a[4];
    }
    rx.assign(size_t(std::max(M, 1)) * kRxInt, 0);
    rk.assign(size_t(std::max(M, 1)) * kRxDbl, 0.0);
    eff.assign(size_t(std::max(M, 1)) * K, 1.0);
    nu.assign(size_t(std::max(M, 1)) * K, 0);
    for (int jd = 0; jd < M; ++jd) {
        const int j = order[jd];  // source reaction stored at device position jd
        int *ri = &rx[size_t(jd) * kRxInt];
        double *rd = &rk[size_t(jd) * kRxDbl];
        ri[0] = m.type[j];
        int nr = 0, np = 0, dnu = 0;
        for (int k = 0; k < K; ++k) {
            for (int c = 0; c < m.nu_r[j * K + k]; ++c) ri[1 + nr++] = 1 + k;
            for (int c = 0; c < m.nu_p[j * K + k]; ++c) ri[4 + np++] = 1 + k;
            dnu += m.nu_p[j * K + k] - m.nu_r[j * K + k];
        }
        ri[7] = dnu;
        rd[0] = std::log(m.arr[3 * j]);
        rd[1] = m.arr[3 * j + 1];
        rd[2] = m.arr[3 * j + 2];
        if (m.type[j] == 2) {
            rd[3] = std::log(m.low[3 * j]);
            rd[4] = m.low[3 * j + 1];
            rd[5] = m.low[3 * j + 2];
            rd[6] = m.troe[4 * j];
            rd[7] = 1.0 / m.troe[4 * j + 1];
            rd[8] = 1.0 / m.troe[4 * j + 2];
            rd[9] = m.troe[4 * j + 3];
        }
        rd[10] = nr;
        rd[11] = np;
        for (int k = 0; k < K; ++k) {
            eff[size_t(jd) * K + k] = m.eff[size_t(j) * K + k];
            nu[size_t(jd) * K + k] = m.nu_p[size_t(j) * K + k] - m.nu_r[size_t(j) * K + k];
        }
    }
    // per-species lists of the reactions that change it
    std::vector<std::vector<std::pair<int, int>>> lists(K);
    for (int j = 0; j < M; ++j)
        for (int k = 0; k < K; ++k)
            if (nu[size_t(j) * K + k] != 0) lists[k].push_back({j, nu[size_t(j) * K + k]});
    lmax = 1;
    for (auto &l : lists) lmax = std::max<int>(lmax, int(l.size()));
    spl.assign(size_t(K) * lmax * 2, 0);
    for (int k = 0; k < K; ++k)
        for (int e = 0; e < lmax; ++e) {
            const bool have = e < int(lists[k].size());
            spl[(size_t(k) * lmax + e) * 2] = have ? lists[k][e].first : M;  // padding: slot M holds zeros
            spl[(size_t(k) * lmax + e) * 2 + 1] = have ? lists[k][e].second : 0;
        }
}

df_status validate_chem_opts(const df_chem_opts &o) {
    if (!(o.rtol > 0 && o.rtol < 1) || !(o.atol_T > 0) || !(o.atol_Y > 0) || !(o.h_min > 0) || o.max_steps < 1 ||
        o.mapping < 0 || o.mapping > 2 || !std::isfinite(o.atol_T) || !std::isfinite(o.atol_Y) ||
        !std::isfinite(o.h_min))
        return fail(DF_E_INVALID, "df_chem_opts: need 0 < rtol < 1, atol_T, atol_Y, h_min > 0 and finite, "
                                  "max_steps >= 1, mapping in {0, 1, 2}");
    return DF_OK;
}

}  // namespace df

using namespace df;

extern "C" {

const char *df_last_error(void) { return g_last_error.c_str(); }

const char *df_version(void) { return "df-mi355x 0.1 (gfx950)"; }

void df_chem_default_opts(df_chem_opts *o) {
    if (!o) return;
    o->rtol = 1e-8;
    o->atol_T = 1e-6;
    o->atol_Y = 1e-14;
    o->h_min = 1e-20;
    o->max_steps = 100000;
    o->mapping = 0;
}

void df_dnn_default_opts(df_dnn_opts *o) {
    if (!o) return;
    o->renormalise = 1;
    o->fallback = 1;
    o->reserved0 = 0;
    o->reserved1 = 0;
}

df_status df_mech_load(const char *path, int32_t device, df_mech **out) {
    clear_error();
    if (!path || !out) return fail(DF_E_INVALID, "df_mech_load: null path or out");
    *out = nullptr;
    HostMech hm;
    df_status st = parse_mech_file(path, hm);
    if (st != DF_OK) return st;
    std::vector<double> sp, rk, eff;
    std::vector<int> rx, nu, spl;
    int lmax = 1;
    pack_tables(hm, sp, rx, rk, eff, nu, spl, lmax);
    // one allocation: [sp | rk | eff | rx | nu | spl], each part 256-byte aligned
    auto align = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t o_sp = 0, o_rk = align(o_sp + sp.size() * 8), o_eff = align(o_rk + rk.size() * 8),
           o_rx = align(o_eff + eff.size() * 8), o_nu = align(o_rx + rx.size() * 4),
           o_spl = align(o_nu + nu.size() * 4), total = align(o_spl + spl.size() * 4);
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, "df_mech_load: hipGetDevice failed");
    if (hipSetDevice(device) != hipSuccess) return fail(DF_E_INVALID, "df_mech_load: invalid device");
    void *blob = nullptr;
    hipError_t e = hipMalloc(&blob, total);
    if (e == hipSuccess) {
        std::vector<unsigned char> h(total, 0);
        std::memcpy(h.data() + o_sp, sp.data(), sp.size() * 8);
        std::memcpy(h.data() + o_rk, rk.data(), rk.size() * 8);
        std::memcpy(h.data() + o_eff, eff.data(), eff.size() * 8);
        std::memcpy(h.data() + o_rx, rx.data(), rx.size() * 4);
        std::memcpy(h.data() + o_nu, nu.data(), nu.size() * 4);
        std::memcpy(h.data() + o_spl, spl.data(), spl.size() * 4);
        e = hipMemcpy(blob, h.data(), total, hipMemcpyHostToDevice);
    }
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        if (blob) (void)hipFree(blob);
        return fail(DF_E_HIP, std::string("df_mech_load: ") + hipGetErrorString(e));
    }
    auto *m = new df_mech;
    m->device = device;
    m->host = std::move(hm);
    m->dev_blob = blob;
    auto *base = static_cast<unsigned char *>(blob);
    m->dev.K = m->host.K;
    m->dev.M = m->host.M;
    m->dev.sp = reinterpret_cast<const double *>(base + o_sp);
    m->dev.rk = reinterpret_cast<const double *>(base + o_rk);
    m->dev.eff = reinterpret_cast<const double *>(base + o_eff);
    m->dev.rx = reinterpret_cast<const int *>(base + o_rx);
    m->dev.nu = reinterpret_cast<const int *>(base + o_nu);
    m->dev.spl = reinterpret_cast<const int *>(base + o_spl);
    m->dev.lmax = lmax;
    *out = m;
    return DF_OK;
}

void df_mech_free(df_mech *m) {
    if (!m) return;
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(m->device) == hipSuccess) {
        (void)hipFree(m->dev_blob);
        (void)hipSetDevice(prev);
    }
    delete m;
}

df_status df_mech_info(const df_mech *m, int32_t *n_species, int32_t *n_reactions, int32_t *n_elements) {
    clear_error();
    if (!m) return fail(DF_E_INVALID, "df_mech_info: null handle");
    if (n_species) *n_species = m->host.K;
    if (n_reactions) *n_reactions = m->host.M;
    if (n_elements) *n_elements = m->host.E;
    return DF_OK;
}

}  // extern "C"
