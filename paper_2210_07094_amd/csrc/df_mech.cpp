// Mechanism loading: "dfmech 1" parser, device-table packing, handle lifetime,
// error reporting and option helpers of the C ABI.
#include <algorithm>
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

// Order in which the reactions are stored on the device: falloff rows first, then
// third-body rows, then the rest (stable within each type).  The cooperative kernel
// evaluates stored reaction j on lane j % 16 in slot j / 16, and a wave runs the code
// of a reaction type in a slot only if one of its lanes holds that type there; grouping
// the types keeps the falloff code (several transcendentals) out of all but the first
// slots.  Results do not depend on the order beyond the summation order of rates.
static std::vector<int> device_order(const HostMech &m) {
    std::vector<int> order(m.M);
    for (int j = 0; j < m.M; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return m.type[a] > m.type[b]; });
    return order;
}

// Tables of the one-cell-per-lane kernel (layout in df_internal.h).
static void pack_tables(const HostMech &m, const std::vector<int> &order, std::vector<double> &sp,
                        std::vector<int> &rx, std::vector<double> &rk, std::vector<double> &eff,
                        std::vector<int> &nu) {
    const int K = m.K, M = m.M;
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
}

// Tables of the cooperative kernel (layout in df_internal.h).  The equilibrium constant
// and the reaction enthalpy are linear in the NASA-7 coefficients, so each reaction gets
// its own coefficient rows over a few functions of T: with
//   H_k/(R T) = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T,
//   S_k/R     = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7,
//   g_k = H_k/(R T) - S_k/R,  1/K_c = exp(sum_k nu_k g_k) (p0/(R T))^(-dnu)  [mol/cm^3],
// ln k_r = ln k_f + ln(1/K_c) is one dot product, and so is sum_k nu_k H_k/(R T).
struct CoopTables {
    int RPL = 1, MP = 16, lmax = 0;
    std::vector<double> cr, ceff, ceffw, clc, wlc;
    std::vector<int> ci, cli, wlo, wlj;
};

static void pack_coop_tables(const HostMech &m, const std::vector<int> &order, CoopTables &t) {
    const int K = m.K, M = m.M;
    t.RPL = std::max(1, (M + kCoopLanes - 1) / kCoopLanes);
    t.MP = kCoopLanes * t.RPL;
    const int MP = t.MP, KE = K + 4;
    t.cr.assign(size_t(MP) * kCrDbl, 0.0);
    t.ci.assign(size_t(MP) * kCiInt, 0);
    t.ceff.assign(size_t(MP) * KE, 0.0);
    t.ceffw.assign(size_t(MP) * K, 0.0);
    const double lncref0 = std::log(1e-6 * kPref / kR);  // ln(p0/(R T)) + ln T, mol/cm^3
    std::vector<std::vector<std::pair<int, int>>> lists(K);
    for (int jd = 0; jd < MP; ++jd) {
        int *ri = &t.ci[size_t(jd) * kCiInt];
        for (int e = 0; e < kCoopEnt; ++e) ri[7 + 2 * e] = K + 3;  // unused entries: scratch column
        if (jd >= M) continue;  // inert padding row: all coefficients zero, empty slots
        const int j = order[jd];
        double *cr = &t.cr[size_t(jd) * kCrDbl];
        int nr = 0, np = 0, dnu = 0;
        for (int k = 0; k < K; ++k) {
            for (int c = 0; c < m.nu_r[j * K + k]; ++c) ri[1 + nr++] = 1 + k;
            for (int c = 0; c < m.nu_p[j * K + k]; ++c) ri[4 + np++] = 1 + k;
            dnu += m.nu_p[j * K + k] - m.nu_r[j * K + k];
        }
        ri[0] = m.type[j];
        // distinct species and the slots they occupy
        int ne = 0;
        for (int s = 0; s < 6; ++s) {
            const int sp = ri[1 + s];
            if (sp == 0) continue;
            int e = 0;
            while (e < ne && ri[7 + 2 * e] != sp - 1) ++e;
            if (e == ne) {
                ri[7 + 2 * e] = sp - 1;
                ri[8 + 2 * e] = 0;
                ++ne;
            }
            ri[8 + 2 * e] |= 1 << s;
        }
        double snu[7] = {0, 0, 0, 0, 0, 0, 0};  // sum_k nu_k a_i
        for (int k = 0; k < K; ++k) {
            const int n = m.nu_p[j * K + k] - m.nu_r[j * K + k];
            for (int i = 0; i < 7; ++i) snu[i] += n * m.nasa[7 * k + i];
            if (n != 0) lists[k].push_back({jd, n});
        }
        const double lnA = std::log(m.arr[3 * j]), b = m.arr[3 * j + 1], Ta = m.arr[3 * j + 2];
        cr[0] = lnA;
        cr[1] = b;
        cr[2] = -Ta;
        cr[3] = lnA + snu[0] - snu[6] - dnu * lncref0;
        cr[4] = b - snu[0] + dnu;
        cr[5] = -Ta + snu[5];
        cr[6] = -snu[1] / 2;
        cr[7] = -snu[2] / 6;
        cr[8] = -snu[3] / 12;
        cr[9] = -snu[4] / 20;
        cr[10] = snu[0];
        cr[11] = snu[1] / 2;
        cr[12] = snu[2] / 3;
        cr[13] = snu[3] / 4;
        cr[14] = snu[4] / 5;
        cr[15] = snu[5];
        if (m.type[j] == 2) {
            cr[16] = std::log(m.low[3 * j]) - lnA;
            cr[17] = m.low[3 * j + 1] - b;
            cr[18] = -(m.low[3 * j + 2] - Ta);
            cr[19] = m.troe[4 * j];
            cr[20] = -1.0 / m.troe[4 * j + 1];
            cr[21] = -1.0 / m.troe[4 * j + 2];
            cr[22] = -m.troe[4 * j + 3];
        }
        cr[23] = nr;
        cr[24] = np;
        if (m.type[j] != 0)
            for (int k = 0; k < K; ++k) {
                t.ceff[size_t(jd) * KE + k] = m.eff[size_t(j) * K + k];
                t.ceffw[size_t(jd) * K + k] = m.eff[size_t(j) * K + k] / m.W[k];
            }
    }
    // per-lane lists over the per-cell rate array [q_0 .. q_{MP-1}, 0, partial sums of lanes 0..15]:
    // species lanes 1..K sum nu q over their reactions, lane 0 sums the 16 partial enthalpy sums
    t.lmax = 0;
    for (auto &l : lists) t.lmax = std::max<int>(t.lmax, int(l.size()));
    // the same lists as CSR (packed for the one-wave-per-cell kernel by pack_wave_tables)
    t.wlo.assign(size_t(K) + 1, 0);
    t.wlj.clear();
    t.wlc.clear();
    for (int k = 0; k < K; ++k) {
        for (auto &e : lists[k]) {
            t.wlj.push_back(e.first);
            t.wlc.push_back(double(e.second));
        }
        t.wlo[size_t(k) + 1] = int(t.wlj.size());
    }
    if (t.wlj.empty()) {  // keep every table part non-empty
        t.wlj.push_back(0);
        t.wlc.push_back(0.0);
    }
    t.cli.assign(size_t(kCoopLanes) * kCoopList, MP);
    t.clc.assign(size_t(kCoopLanes) * kCoopList, 0.0);
    for (int e = 0; e < kCoopList; ++e) {
        t.cli[e] = MP + 1 + e;
        t.clc[e] = 1.0;
    }
    for (int k = 0; k < K && k + 1 < kCoopLanes; ++k)
        for (int e = 0; e < std::min<int>(kCoopList, int(lists[k].size())); ++e) {
            t.cli[size_t(k + 1) * kCoopList + e] = lists[k][e].first;
            t.clc[size_t(k + 1) * kCoopList + e] = lists[k][e].second;
        }
}

// Tables of the one-wave-per-cell kernel (layout in df_internal.h), from the coop rows of the
// first M stored reactions: column-major copies (lane t reads field f of reaction t at f M + t,
// so a wave's loads are contiguous), the Jacobian's sparse entries grouped by target in rounds
// of 64 targets, the per-species reaction lists and the third-body reactions of each species row,
// each entry packed into one int.
struct WaveTables {
    std::vector<double> cr, eff;
    std::vector<int> ci, tk, ell, rb, rc, lo, lp, dof, dp;
    int sr = 0, sp = 0;  // reactant and product slots in use
};

// an entry (index < 2^20, small signed coefficient) packed into one int
static int pack_entry(int idx, int nu) { return idx | ((nu + 8) << 20); }

static void pack_wave_tables(const HostMech &m, const CoopTables &ct, WaveTables &w) {
    const int K = m.K, M = m.M, KE = K + 4, LDJ = K + 2;
    w.cr.assign(size_t(kCrDbl) * M, 0.0);
    w.ci.assign(size_t(7) * M, 0);
    w.eff.assign(size_t(K) * M, 0.0);
    for (int jd = 0; jd < M; ++jd) {
        for (int f = 0; f < kCrDbl; ++f) w.cr[size_t(f) * M + jd] = ct.cr[size_t(jd) * kCrDbl + f];
        for (int f = 0; f < 7; ++f) w.ci[size_t(f) * M + jd] = ct.ci[size_t(jd) * kCiInt + f];
        for (int k = 0; k < K; ++k) w.eff[size_t(k) * M + jd] = ct.ceff[size_t(jd) * KE + k];
    }
    // sparse part: J(1 + k, 1 + l) = sum over reactions jd containing k and l of
    // nu_k(jd) * (derivative of q_jd with respect to the concentration in each slot holding l)
    // slots in use (reactant slots fill 0, 1, 2 and product slots 3, 4, 5 in order); the slot
    // derivatives keep one row per slot in use
    w.sr = w.sp = 0;
    for (int jd = 0; jd < M; ++jd)
        for (int s = 0; s < 3; ++s) {
            if (ct.ci[size_t(jd) * kCiInt + 1 + s] != 0) w.sr = std::max(w.sr, s + 1);
            if (ct.ci[size_t(jd) * kCiInt + 4 + s] != 0) w.sp = std::max(w.sp, s + 1);
        }
    auto drow = [&](int s) { return s < 3 ? s : w.sr + (s - 3); };
    std::vector<std::vector<std::pair<int, int>>> ent(size_t(K) * K);
    for (int jd = 0; jd < M; ++jd) {
        const int *ri = &ct.ci[size_t(jd) * kCiInt];
        for (int a = 0; a < kCoopEnt; ++a) {
            const int k = ri[7 + 2 * a];
            if (k >= K) continue;
            const int mk = ri[8 + 2 * a];
            int nuk = 0;
            for (int s = 0; s < 6; ++s)
                if (mk & (1 << s)) nuk += (s < 3) ? -1 : 1;
            for (int b = 0; b < kCoopEnt; ++b) {
                const int l = ri[7 + 2 * b];
                if (l >= K) continue;
                const int ml = ri[8 + 2 * b];
                for (int s = 0; s < 6; ++s)
                    if (ml & (1 << s)) ent[size_t(k) * K + l].push_back({drow(s) * M + jd, nuk});
            }
        }
    }
    // targets in rounds of 64 (one per lane); a round's entries column-major (entry e of lane l
    // at rb[r] + 64 e + l), padded with coefficient-0 entries to the round's longest list rc[r].
    // Targets are taken longest list first, so a round's lists are of similar length (in
    // (k, l) order the long diagonal lists would pad every round: 11x the entries instead of
    // 1.3x for the 53-species mechanism).
    std::vector<const std::vector<std::pair<int, int>> *> lt;
    std::vector<int> tk0;
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) {
            const auto &e = ent[size_t(k) * K + l];
            if (e.empty()) continue;
            tk0.push_back((1 + k) * LDJ + 1 + l);
            lt.push_back(&e);
        }
    {
        std::vector<int> ord(lt.size());
        for (size_t i = 0; i < ord.size(); ++i) ord[i] = int(i);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return lt[a]->size() > lt[b]->size(); });
        std::vector<const std::vector<std::pair<int, int>> *> lt2;
        w.tk.clear();
        for (int i : ord) {
            lt2.push_back(lt[i]);
            w.tk.push_back(tk0[i]);
        }
        lt.swap(lt2);
    }
    const int NT = int(w.tk.size());
    w.ell.clear();
    w.rb.clear();
    w.rc.clear();
    for (int r = 0; r * 64 < NT; ++r) {
        int cm = 0;
        for (int l = 0; l < 64 && r * 64 + l < NT; ++l) cm = std::max<int>(cm, int(lt[r * 64 + l]->size()));
        w.rb.push_back(int(w.ell.size()));
        w.rc.push_back(cm);
        for (int e = 0; e < cm; ++e)
            for (int l = 0; l < 64; ++l) {
                const int t = r * 64 + l;
                const bool has = t < NT && e < int(lt[t]->size());
                w.ell.push_back(has ? pack_entry((*lt[t])[e].first, (*lt[t])[e].second) : pack_entry(0, 0));
            }
    }
    // the per-species reaction lists, packed (reaction, nu)
    w.lo = ct.wlo;
    w.lp.clear();
    for (size_t e = 0; e < ct.wlj.size(); ++e) w.lp.push_back(pack_entry(ct.wlj[e], int(ct.wlc[e])));
    // dense third-body part, per species row k: the third-body and falloff reactions with nu_k != 0
    w.dof.assign(size_t(K) + 1, 0);
    w.dp.clear();
    for (int k = 0; k < K; ++k) {
        for (int jd = 0; jd < M; ++jd) {
            const int *ri = &ct.ci[size_t(jd) * kCiInt];
            if (ri[0] == 0) continue;
            int nuk = 0;
            for (int s = 0; s < 6; ++s)
                if (ri[1 + s] == 1 + k) nuk += (s < 3) ? -1 : 1;
            if (nuk != 0) w.dp.push_back(pack_entry(jd, nuk));
        }
        w.dof[size_t(k) + 1] = int(w.dp.size());
    }
    // keep every table part non-empty
    if (w.cr.empty()) w.cr.push_back(0.0);
    if (w.ci.empty()) w.ci.push_back(0);
    if (w.eff.empty()) w.eff.push_back(0.0);
    if (w.tk.empty()) w.tk.push_back(0);
    if (w.ell.empty()) w.ell.push_back(pack_entry(0, 0));
    if (w.rb.empty()) {
        w.rb.push_back(0);
        w.rc.push_back(0);
    }
    if (w.lp.empty()) w.lp.push_back(pack_entry(0, 0));
    if (w.dp.empty()) w.dp.push_back(pack_entry(0, 0));
}

df_status validate_chem_opts(const df_chem_opts &o) {
    if (!(o.rtol > 0 && o.rtol < 1) || !(o.atol_T > 0) || !(o.atol_Y > 0) || !(o.h_min > 0) || o.max_steps < 1 ||
        o.mapping < 0 || o.mapping > 5 || o.schedule < 0 || o.schedule > 2 || o.coop_blocks < -1 ||
        !std::isfinite(o.atol_T) || !std::isfinite(o.atol_Y) || !std::isfinite(o.h_min))
        return fail(DF_E_INVALID, "df_chem_opts: need 0 < rtol < 1, atol_T, atol_Y, h_min > 0 and finite, "
                                  "max_steps >= 1, mapping in {0, 1, 2, 3, 4, 5}, schedule in {0, 1, 2}, coop_blocks >= -1");
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
    o->schedule = 0;
    o->coop_blocks = 0;
}

void df_dnn_default_opts(df_dnn_opts *o) {
    if (!o) return;
    o->renormalise = 1;
    o->fallback = 1;
    o->precision = 0;
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
    std::vector<int> rx, nu;
    const std::vector<int> order = device_order(hm);
    pack_tables(hm, order, sp, rx, rk, eff, nu);
    CoopTables ct;
    pack_coop_tables(hm, order, ct);
    WaveTables wt;
    pack_wave_tables(hm, ct, wt);
    // one allocation holding every table, each part 256-byte aligned
    struct Part {
        const void *src;
        size_t bytes, off;
    };
    Part parts[] = {{sp.data(), sp.size() * 8, 0},          {rk.data(), rk.size() * 8, 0},
                    {eff.data(), eff.size() * 8, 0},        {rx.data(), rx.size() * 4, 0},
                    {nu.data(), nu.size() * 4, 0},          {ct.cr.data(), ct.cr.size() * 8, 0},
                    {ct.ci.data(), ct.ci.size() * 4, 0},    {ct.ceff.data(), ct.ceff.size() * 8, 0},
                    {ct.ceffw.data(), ct.ceffw.size() * 8, 0}, {ct.cli.data(), ct.cli.size() * 4, 0},
                    {ct.clc.data(), ct.clc.size() * 8, 0},  {order.data(), order.size() * 4, 0},
                    {wt.cr.data(), wt.cr.size() * 8, 0},
                    {wt.ci.data(), wt.ci.size() * 4, 0},    {wt.eff.data(), wt.eff.size() * 8, 0},
                    {wt.tk.data(), wt.tk.size() * 4, 0},    {wt.ell.data(), wt.ell.size() * 4, 0},
                    {wt.rb.data(), wt.rb.size() * 4, 0},    {wt.rc.data(), wt.rc.size() * 4, 0},
                    {wt.lo.data(), wt.lo.size() * 4, 0},    {wt.lp.data(), wt.lp.size() * 4, 0},
                    {wt.dof.data(), wt.dof.size() * 4, 0},  {wt.dp.data(), wt.dp.size() * 4, 0}};
    size_t total = 0;
    for (auto &q : parts) {
        q.off = total;
        total = (total + q.bytes + 255) & ~size_t(255);
    }
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, "df_mech_load: hipGetDevice failed");
    if (hipSetDevice(device) != hipSuccess) return fail(DF_E_INVALID, "df_mech_load: invalid device");
    void *blob = nullptr;
    hipError_t e = hipMalloc(&blob, total);
    if (e == hipSuccess) {
        std::vector<unsigned char> h(total, 0);
        for (auto &q : parts) std::memcpy(h.data() + q.off, q.src, q.bytes);
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
    auto D = [&](int i) { return reinterpret_cast<const double *>(base + parts[i].off); };
    auto I = [&](int i) { return reinterpret_cast<const int *>(base + parts[i].off); };
    m->dev.K = m->host.K;
    m->dev.M = m->host.M;
    m->dev.sp = D(0);
    m->dev.rk = D(1);
    m->dev.eff = D(2);
    m->dev.rx = I(3);
    m->dev.nu = I(4);
    m->dev.RPL = ct.RPL;
    m->dev.lmax = ct.lmax;
    m->dev.cr = D(5);
    m->dev.ci = I(6);
    m->dev.ceff = D(7);
    m->dev.ceffw = D(8);
    m->dev.cli = I(9);
    m->dev.clc = D(10);
    m->dev.src = I(11);
    m->dev.wcr = D(12);
    m->dev.wci = I(13);
    m->dev.weff = D(14);
    m->dev.wtk = I(15);
    m->dev.well = I(16);
    m->dev.wrb = I(17);
    m->dev.wrc = I(18);
    m->dev.wlo = I(19);
    m->dev.wlp = I(20);
    m->dev.wdo = I(21);
    m->dev.wdp = I(22);
    m->dev.wnr = int(wt.rb.size());
    m->dev.wsr = wt.sr;
    m->dev.wsp = wt.sp;
    m->dev.wnt = m->dev.wnr > 0 && wt.rc[0] > 0 ? int(wt.tk.size()) : 0;
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
