// k_const.hip -- host tables and launches of the constant-coefficient line
// solves (strided y / z lines, staged x lines, and the ADI stencil + x solve).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "const_lines.hpp"
#include "dispatch.hpp"

namespace trid {

template <typename T>
bool make_const_tab(double a, double b, double c, int M, int P, ConstTab<T> *t) {
    if (M < 3 || M > kConstMaxM || P < 1 || P > kConstMaxP) return false;
    std::memset(static_cast<void *>(t), 0, sizeof(*t));
    // coefficient part of the tile sweep (eq. (7)) on rows (a, b, c)
    double rr[kConstMaxM] = {0}, apf[kConstMaxM] = {0}, cpf[kConstMaxM] = {0};
    rr[1] = 1.0 / b;
    apf[1] = a * rr[1];
    cpf[1] = c * rr[1];
    for (int k = 2; k < M; ++k) {
        rr[k] = 1.0 / (b - a * cpf[k - 1]);
        apf[k] = -rr[k] * a * apf[k - 1];
        cpf[k] = rr[k] * c;
    }
    double ap[kConstMaxM], cp[kConstMaxM];
    std::memcpy(ap, apf, sizeof ap);
    std::memcpy(cp, cpf, sizeof cp);
    for (int k = M - 3; k >= 1; --k) {
        ap[k] -= cp[k] * ap[k + 1];
        cp[k] = -cp[k] * cp[k + 1];
    }
    const double la = apf[M - 1], lc = cpf[M - 1];
    const double fb = b - c * ap[1], fc = -c * cp[1];
    for (int k = 0; k < M; ++k) {
        t->rr[k] = (T)rr[k];
        t->am[k] = (T)(rr[k] * a);
        t->cpf[k] = (T)cpf[k];
        t->apb[k] = (T)ap[k];
        t->cpb[k] = (T)cp[k];
    }
    t->c = (T)c;
    t->la = (T)la;
    t->lc = (T)lc;
    t->P = P;
    // reduced system over the tiles' first unknowns: G f = fd - fa*ld_{p-1} - fc*ld_p
    double G[kConstMaxP][kConstMaxP] = {{0}}, inv[kConstMaxP][kConstMaxP] = {{0}};
    auto fa = [&](int p) { return p == 0 ? 0.0 : a; };
    auto lcp = [&](int p) { return p == P - 1 ? 0.0 : lc; };
    for (int p = 0; p < P; ++p) {
        if (p > 0) G[p][p - 1] = -fa(p) * la;
        G[p][p] = fb - fa(p) * (p > 0 ? lcp(p - 1) : 0.0) - fc * la;
        if (p + 1 < P) G[p][p + 1] = -fc * lcp(p);
        inv[p][p] = 1.0;
    }
    // Gauss-Jordan with partial pivoting (P <= 8)
    for (int col = 0; col < P; ++col) {
        int piv = col;
        for (int r = col + 1; r < P; ++r)
            if (std::fabs(G[r][col]) > std::fabs(G[piv][col])) piv = r;
        if (G[piv][col] == 0.0) return false;
        for (int k = 0; k < P; ++k) {
            std::swap(G[col][k], G[piv][k]);
            std::swap(inv[col][k], inv[piv][k]);
        }
        const double rp = 1.0 / G[col][col];
        for (int k = 0; k < P; ++k) {
            G[col][k] *= rp;
            inv[col][k] *= rp;
        }
        for (int r = 0; r < P; ++r) {
            if (r == col || G[r][col] == 0.0) continue;
            const double f = G[r][col];
            for (int k = 0; k < P; ++k) {
                G[r][k] -= f * G[col][k];
                inv[r][k] -= f * inv[col][k];
            }
        }
    }
    for (int p = 0; p < P; ++p)
        for (int q = 0; q < P; ++q) {
            t->w1[p * kConstMaxP + q] = (T)inv[p][q];
            const double nxt = (q + 1 < P) ? fa(q + 1) * inv[p][q + 1] : 0.0;
            t->w2[p * kConstMaxP + q] = (T)(-fc * inv[p][q] - nxt);
        }
    return true;
}

template bool make_const_tab<double>(double, double, double, int, int, ConstTab<double> *);
template bool make_const_tab<float>(double, double, double, int, int, ConstTab<float> *);

template <typename T>
bool make_pcr_tab(double a, double b, double c, int M, int P, PcrTab<T> *t) {
    if (P < 1 || P > kDppMaxP) return false;
    ConstTab<T> ct;
    if (!make_const_tab<T>(a, b, c, M, 1, &ct)) return false;  // tile tables (P = 1: no W needed)
    std::memset(static_cast<void *>(t), 0, sizeof(*t));
    std::memcpy(t->rr, ct.rr, sizeof t->rr);
    std::memcpy(t->am, ct.am, sizeof t->am);
    std::memcpy(t->cpf, ct.cpf, sizeof t->cpf);
    std::memcpy(t->apb, ct.apb, sizeof t->apb);
    std::memcpy(t->cpb, ct.cpb, sizeof t->cpb);
    t->c = ct.c;
    t->la = ct.la;
    t->lc = ct.lc;
    // recompute the first-row factors in FP64 (the tables above are rounded to T)
    double cpf[kConstMaxM] = {0}, apf[kConstMaxM] = {0}, rr[kConstMaxM] = {0};
    rr[1] = 1.0 / b;
    apf[1] = a * rr[1];
    cpf[1] = c * rr[1];
    for (int k = 2; k < M; ++k) {
        rr[k] = 1.0 / (b - a * cpf[k - 1]);
        apf[k] = -rr[k] * a * apf[k - 1];
        cpf[k] = rr[k] * c;
    }
    double ap[kConstMaxM], cp[kConstMaxM];
    std::memcpy(ap, apf, sizeof ap);
    std::memcpy(cp, cpf, sizeof cp);
    for (int k = M - 3; k >= 1; --k) {
        ap[k] -= cp[k] * ap[k + 1];
        cp[k] = -cp[k] * cp[k + 1];
    }
    const double la = apf[M - 1], lc = cpf[M - 1];
    const double fb = b - c * ap[1], fc = -c * cp[1];
    double ga[kDppMaxP] = {0}, gc[kDppMaxP] = {0};
    for (int p = 0; p < P; ++p) {
        const double fa = p == 0 ? 0.0 : a;
        const double lcm = p == 0 ? 0.0 : (p - 1 == P - 1 ? 0.0 : lc);
        const double lcp = p == P - 1 ? 0.0 : lc;
        const double dia = fb - fa * lcm - fc * la;
        if (dia == 0.0) return false;
        const double rg = 1.0 / dia;
        ga[p] = -fa * la * rg;
        gc[p] = -fc * lcp * rg;
        t->rg[p] = (T)rg;
        t->gA[p] = (T)(fa * rg);
        t->gC[p] = (T)(fc * rg);
    }
    for (int j = 0, s = 1; s < P; ++j, s *= 2) {
        double na[kDppMaxP], nc[kDppMaxP];
        for (int p = 0; p < P; ++p) {
            const double am = p - s >= 0 ? ga[p - s] : 0.0, cm = p - s >= 0 ? gc[p - s] : 0.0;
            const double an = p + s < P ? ga[p + s] : 0.0, cn = p + s < P ? gc[p + s] : 0.0;
            const double den = 1.0 - ga[p] * cm - gc[p] * an;
            if (den == 0.0) return false;
            const double r = 1.0 / den;
            t->pr[j][p] = (T)r;
            t->pa[j][p] = (T)(r * ga[p]);
            t->pc[j][p] = (T)(r * gc[p]);
            na[p] = -r * ga[p] * am;
            nc[p] = -r * gc[p] * cn;
        }
        std::memcpy(ga, na, sizeof(double) * P);
        std::memcpy(gc, nc, sizeof(double) * P);
    }
    return true;
}

namespace {

i64 cdiv(i64 a, i64 b) { return (a + b - 1) / b; }

template <typename T, int M, class Epi>
hipError_t go_strided(const LineReq &r, const ConstTab<T> &tb, Epi epi, hipStream_t s) {
    StridedGeom g;
    g.inner = r.inner;
    g.nib = cdiv(r.inner, 64);
    g.n = (int)r.n;
    g.L = 64;
    g.P = tb.P;
    g.lines = (unsigned)(r.inner * r.outer);
    const i64 nb = cdiv(r.inner * r.outer, 64);
    launch((k_strided_const<T, M, Epi>), dim3((unsigned)nb), dim3(64 * tb.P), 0, s, g, tb,
                       static_cast<const T *>(r.d), epi);
    return hipGetLastError();
}

template <typename T, int M, int P, class Src>
hipError_t go_dpp(i64 nlines, int n, const PcrTab<T> &tb, Src src, T *out, int force_L, hipStream_t s) {
    ConstStagedGeom g;
    g.nlines = nlines;
    g.n = n;
    // 128-thread blocks for FP64 (measured faster than 256 on the 256^3 step),
    // 256 for FP32.  A forced line count is taken when the block stays a whole
    // number of wavefronts of at most 256 threads (the staging maps a line row
    // onto at most one wavefront).
    int nt = (sizeof(T) == 8 && n / 2 <= 128) ? 128 : 256;
    if (force_L > 0 && force_L * P <= 256 && (force_L * P) % 64 == 0) nt = force_L * P;
    g.L = nt / P;
    g.ls = P * (M + 1);
    src.block_order(g);
    const size_t shm = (size_t)g.L * g.ls * sizeof(T) + (size_t)g.L * sizeof(int);
    launch((k_staged_dpp<T, M, P, Src>), dim3((unsigned)cdiv(nlines, g.L)), dim3(g.L * P),
                       shm, s, g, tb, src, out);
    return hipGetLastError();
}

// Lines of P in {3, 5, 6, 7} tiles: 256 threads, L = 4 (64 / P) lines, or
// fewer when the source's thread groups stage fewer (the right-hand-side
// source gives each group of C = n / VB threads LG = M / VB lines, VB = one or
// two 16-byte vectors).
template <typename T, int M, int P, class Src>
hipError_t go_lanes(i64 nlines, int n, const PcrTab<T> &tb, Src src, T *out, int force_L, hipStream_t s) {
    ConstStagedGeom g;
    g.nlines = nlines;
    g.n = n;
    constexpr int V = 16 / (int)sizeof(T);
    const int VB = (n / V > 64 ? 2 : 1) * V;
    int L = 4 * (64 / P);
    L = std::min(L, (256 / (n / VB)) * (M / VB));
    if (force_L > 0 && force_L < L) L = force_L;
    g.L = L;
    g.ls = P * (M + 1);
    src.block_order(g);
    const size_t shm = (size_t)g.L * g.ls * sizeof(T) + (size_t)g.L * sizeof(int);
    launch((k_staged_lanes<T, M, P, Src>), dim3((unsigned)cdiv(nlines, g.L)), dim3(256), shm, s, g, tb, src,
           out);
    return hipGetLastError();
}

template <typename T, int M, class Src>
hipError_t go_dpp_p(i64 nlines, int n, const PcrTab<T> &tb, int P, Src src, T *out, int fl, hipStream_t s) {
    switch (P) {
        case 1: return go_dpp<T, M, 1>(nlines, n, tb, src, out, fl, s);
        case 2: return go_dpp<T, M, 2>(nlines, n, tb, src, out, fl, s);
        case 4: return go_dpp<T, M, 4>(nlines, n, tb, src, out, fl, s);
        case 8: return go_dpp<T, M, 8>(nlines, n, tb, src, out, fl, s);
        case 16: return go_dpp<T, M, 16>(nlines, n, tb, src, out, fl, s);
        case 3: return go_lanes<T, M, 3>(nlines, n, tb, src, out, fl, s);
        case 5: return go_lanes<T, M, 5>(nlines, n, tb, src, out, fl, s);
        case 6: return go_lanes<T, M, 6>(nlines, n, tb, src, out, fl, s);
        case 7: return go_lanes<T, M, 7>(nlines, n, tb, src, out, fl, s);
        default: return hipErrorInvalidValue;
    }
}

// Staged x lines with constant rows: PcrTab + DPP kernel.
template <typename T, class Src>
hipError_t staged_dpp(double a, double b, double c, int M, i64 nlines, int n, Src src, T *out, int force_L,
                      hipStream_t s) {
    PcrTab<T> tb;
    const int P = n / M;
    if (!make_pcr_tab<T>(a, b, c, M, P, &tb)) return hipErrorInvalidValue;
    return M == 32 ? go_dpp_p<T, 32>(nlines, n, tb, P, src, out, force_L, s)
                   : go_dpp_p<T, 16>(nlines, n, tb, P, src, out, force_L, s);
}

template <typename T>
bool aligned16(const void *p) {
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Tile rows for constant rows on strided lines: the largest of 32, 16 dividing
// n with n / M <= 8 (dense reduced inverse).
int const_M(i64 n, int force_M) {
    for (int M : {32, 16}) {
        if (force_M && M != force_M) continue;
        if (n % M == 0 && n / M >= 1 && n / M <= kConstMaxP) return M;
    }
    return 0;
}

// Tile rows for constant rows on staged x lines: P = n / M a power of two <=
// 16 (DPP reduced solve), else P in {3, 5, 6, 7} (whole lines per wavefront,
// lane-move reduced solve); prefer 128 bytes of tile per thread (M w = 128).
int const_staged_M(i64 n, int w, int force_M) {
    // 128-byte tiles first (16 FP64 or 32 FP32 rows), except for FP32 lines of
    // at least 256 points split into a power of two of 16-row tiles (more,
    // shorter tiles measured 7-10% faster there); 3, 5, 6 or 7 tiles keep the
    // 128-byte order
    const int pref[2] = {128 / w, 128 / w == 16 ? 32 : 16};
    const int pref16[2] = {16, 32};
    for (int pass = 0; pass < 2; ++pass) {
        const bool fp32_long = pass == 0 && w == 4 && n >= 256;
        for (int M : fp32_long ? pref16 : pref) {
            if (force_M && M != force_M) continue;
            if (n % M) continue;
            const i64 P = n / M;
            if (pass == 0 && P >= 1 && P <= kDppMaxP && (P & (P - 1)) == 0) return M;
            if (pass == 1 && (P == 3 || P == 5 || P == 6 || P == 7)) return M;
        }
    }
    return 0;
}

template <typename T>
hipError_t lines_typed(const LineReq &r, int M, hipStream_t s) {
    if (r.inner == 1) {
        CStgCopy<T> src{static_cast<const T *>(r.d)};
        return staged_dpp<T>(r.ca, r.cb, r.cc, M, r.outer, (int)r.n, src, static_cast<T *>(r.x), r.force_L, s);
    }
    ConstTab<T> tb;
    if (!make_const_tab<T>(r.ca, r.cb, r.cc, M, (int)(r.n / M), &tb)) return hipErrorInvalidValue;
    T *x = static_cast<T *>(r.x);
    if (r.out == Out::Add)
        return M == 32 ? go_strided<T, 32>(r, tb, EpiAdd<T>{x}, s) : go_strided<T, 16>(r, tb, EpiAdd<T>{x}, s);
    return M == 32 ? go_strided<T, 32>(r, tb, EpiStore<T>{x}, s) : go_strided<T, 16>(r, tb, EpiStore<T>{x}, s);
}

template <typename T>
hipError_t rhs_typed(const AdiReq &r, int M, hipStream_t s) {
    const i64 nlines = r.ny * r.nz * r.batch;
    T *out = static_cast<T *>(r.d);
    const T *u = static_cast<const T *>(r.u);
    const double a = -r.s0, b = 1.0 + 2.0 * r.s0, c = -r.s0;
    if (r.ndim == 3) {
        CStgRhs<T, 3> src{u, (T)(2.0 * r.s0), (int)r.ny, (int)r.nz};
        return staged_dpp<T>(a, b, c, M, nlines, (int)r.nx, src, out, r.force_L, s);
    }
    CStgRhs<T, 2> src{u, (T)(2.0 * r.s0), (int)r.ny, 1};
    return staged_dpp<T>(a, b, c, M, nlines, (int)r.nx, src, out, r.force_L, s);
}

}  // namespace

int const_lines_M(const LineReq &r) {
    if (r.mode != Mode::Const || (r.out != Out::Store && r.out != Out::Add)) return 0;
    if (r.inner == 1 && r.out != Out::Store) return 0;
    if (r.n * r.inner >= ((i64)1 << 31)) return 0;  // 32-bit row offsets within a slab
    // 32-bit line numbers: a block's first line plus its lane stays below 2^32
    if (r.inner > 1 && r.inner * r.outer >= ((i64)1 << 31)) return 0;
    const int M = r.inner == 1 ? const_staged_M(r.n, r.f64 ? 8 : 4, r.force_M) : const_M(r.n, r.force_M);
    if (!M) return 0;
    if (r.inner == 1) {
        const int V = r.f64 ? 2 : 4;
        if (r.n % V || !aligned16<char>(r.d) || !aligned16<char>(r.x)) return 0;
    }
    return M;
}

hipError_t launch_const_lines(const LineReq &r, int M, hipStream_t s) {
    return r.f64 ? lines_typed<double>(r, M, s) : lines_typed<float>(r, M, s);
}

int const_rhs_M(const AdiReq &r) {
    if (r.s) return 0;
    // 32-bit line indices and 32-bit byte offsets
    if (r.nx * r.ny * r.nz * r.batch * (r.f64 ? 8 : 4) >= ((i64)1 << 32)) return 0;
    const int M = const_staged_M(r.nx, r.f64 ? 8 : 4, r.force_M);
    if (!M) return 0;
    const int V = r.f64 ? 2 : 4;
    if (r.nx % V || !aligned16<char>(r.u) || !aligned16<char>(r.d)) return 0;
    return M;
}

void const_rhs_geometry(const AdiReq &r, int M, int *threads, int *L, size_t *shmem, i64 *nblocks) {
    const int w = r.f64 ? 8 : 4, n = (int)r.nx, P = n / M;
    int nt = 256, lines;
    if ((P & (P - 1)) == 0) {
        nt = (w == 8 && n / 2 <= 128) ? 128 : 256;
        if (r.force_L > 0 && r.force_L * P <= 256 && (r.force_L * P) % 64 == 0) nt = r.force_L * P;
        lines = nt / P;
    } else {
        const int V = 16 / w, VB = (n / V > 64 ? 2 : 1) * V;
        lines = std::min(4 * (64 / P), (256 / (n / VB)) * (M / VB));
        if (r.force_L > 0 && r.force_L < lines) lines = r.force_L;
    }
    const int ls = P * (M + 1);
    *threads = nt;
    *L = lines;
    *shmem = (size_t)lines * ls * w + (size_t)lines * sizeof(int);
    *nblocks = cdiv(r.ny * r.nz * r.batch, lines);
}

hipError_t launch_const_rhs_x(const AdiReq &r, int M, hipStream_t s) {
    return r.f64 ? rhs_typed<double>(r, M, s) : rhs_typed<float>(r, M, s);
}

}  // namespace trid
