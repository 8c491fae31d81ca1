// k_long.hip -- contiguous lines longer than one workgroup holds (n > TRID_MAX_LINE).
//
// The tiling of Section III-B applied one level up: a line is cut into chunks of
// C = P * M rows, one workgroup per chunk, and every chunk is a "tile" in the
// sense of eq. (7):
//   1. chunk pass: with the chunk's first and last unknowns u_0, u_{C-1} taken
//      as given, the interior solution is s1 + u_0 s2 + u_{C-1} s3, where s1,
//      s2, s3 solve the chunk's rows (first and last replaced by identity rows)
//      with right-hand sides (0, d_1..d_{C-2}, 0), e_0 and e_{C-1}.  Putting
//      rows 1 and C-2 of that into the chunk's original first and last rows
//      gives two reduced rows over (last unknown of the previous chunk, u_0,
//      u_{C-1}, first unknown of the next chunk);
//   2. the 2 * nchunks reduced rows of a line form a tridiagonal system, solved
//      by the batched solver (each line fits one workgroup);
//   3. solve pass: the chunk's rows with its first and last rows replaced by
//      the identity and right-hand sides u_0, u_{C-1} from step 2.
// Reduced systems of diagonally dominant rows stay diagonally dominant (they
// are Schur complements), so no pivoting is introduced.  Traffic: the chunk
// pass reads the rows, the solve pass reads them again and writes x.
#include <algorithm>

#include "lines.hpp"
#include "long_lines.hpp"

namespace trid {

namespace {

constexpr int kM = 8;    // rows per tile
constexpr int kP = 256;  // tiles (threads) per chunk
constexpr int kC = kM * kP;

struct ChunkArgs {
    i64 n;      // line length
    int nch;    // chunks per line
    int ls;     // LDS elements of the staged chunk
    int mode;   // 0 arrays, 1 per-point s, 2 constant rows
    const void *a, *b, *c, *s, *d;
    double ca, cb, cc;
    void *x;
    void *ra, *rb, *rc, *rd;  // reduced rows (chunk pass output)
    const void *rx;           // reduced solution (solve pass input)
};

// Reduced solve (Section III-B, PCR of Alg. 2) of a chunk's P = blockDim.x
// tiles for three right-hand sides sharing one matrix: the first from the
// tile sweep ts, the second and third the unit vectors at the chunk's first and
// last row, which enter only as fd2 (first row of tile 0) and ld3 (last row of
// tile P-1).  sh holds 10 * P elements.  Returns each right-hand side's first
// (f) and last (lv) unknown of this tile.  Every thread of the block calls it.
template <typename T, int M>
__device__ __forceinline__ void reduced_pcr3(const TileState<T, M> &ts, T fd2, T ld3, T *__restrict__ sh,
                                             int p, T (&f)[3], T (&lv)[3]) {
    const int P = blockDim.x;
    constexpr int NA = 5;  // a, c and three right-hand sides per buffer
    T *buf0 = sh, *buf1 = sh + NA * P;
    // previous tile's last row (the second and third right-hand sides are zero
    // there: ld3 is nonzero only on the last tile, which has no successor)
    buf1[p] = ts.la;
    buf1[P + p] = ts.lc;
    buf1[2 * P + p] = ts.ld;
    __syncthreads();
    T pa = T(0), pc = T(0), pd = T(0);
    if (p > 0) {
        pa = buf1[p - 1];
        pc = buf1[P + p - 1];
        pd = buf1[2 * P + p - 1];
    }
    const T rg = fast_rcp(ts.fb - ts.fa * pc - ts.fc * ts.la);
    T a = -ts.fa * pa * rg;
    T c = -ts.fc * ts.lc * rg;
    T d[3] = {(ts.fd - ts.fa * pd - ts.fc * ts.ld) * rg, fd2 * rg, -ts.fc * ld3 * rg};
    int lev = 0;
    for (int s = 1; s < P; s <<= 1, ++lev) {
        T *b = (lev & 1) ? buf1 : buf0;
        b[p] = a;
        b[P + p] = c;
#pragma unroll
        for (int r = 0; r < 3; ++r) b[(2 + r) * P + p] = d[r];
        __syncthreads();
        const bool lo = p - s >= 0, hi = p + s < P;
        const int qm = lo ? p - s : p, qn = hi ? p + s : p;
        const T am = lo ? b[qm] : T(0), cm = lo ? b[P + qm] : T(0);
        const T an = hi ? b[qn] : T(0), cn = hi ? b[P + qn] : T(0);
        const T r = fast_rcp(T(1) - a * cm - c * an);
        T nd[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T dm = lo ? b[(2 + k) * P + qm] : T(0);
            const T dn = hi ? b[(2 + k) * P + qn] : T(0);
            nd[k] = r * (d[k] - a * dm - c * dn);
        }
        const T na = -r * (a * am), nc = -r * (c * cn);
        a = na;
        c = nc;
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = nd[k];
    }
    // the next tile's first unknowns, through the buffer last read two levels ago
    T *b = (lev & 1) ? buf1 : buf0;
#pragma unroll
    for (int k = 0; k < 3; ++k) b[k * P + p] = d[k];
    __syncthreads();
    const bool hi = p + 1 < P;
    const T ld[3] = {ts.ld, T(0), ld3};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T fn = hi ? b[k * P + p + 1] : T(0);
        f[k] = d[k];
        lv[k] = ld[k] - ts.la * d[k] - ts.lc * fn;
    }
}

// Rows of this thread's tile, chunk-local rows g0..g0+M-1; cnt valid rows in
// the chunk; first/last: the chunk holds the line's first / last row.
template <typename T, int PASS>
__global__ __launch_bounds__(kP) void k_chunk(ChunkArgs g) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    // the reduced solve's scratch reuses the staging area: the rows are in
    // registers by then (every put ends with a barrier)
    T *red = sh;
    const int p = threadIdx.x;
    const i64 id = xcd_block_id();
    const i64 line = id / g.nch;
    const int ch = (int)(id - line * g.nch);
    const i64 base = line * g.n + (i64)ch * kC;
    const int cnt = (int)std::min<i64>(kC, g.n - (i64)ch * kC);
    const int g0 = p * kM;
    const int pos = p * (kM + 1);
    T ra[kM], rb[kM], rc[kM], rd[kM];
    // every array's loads are issued before the first is staged, so a block
    // waits for memory once rather than once per array
    auto put = [&](const T(&v)[kM], T(&dst)[kM], T idle) {
        stage_put<T, kM>(sh, v, cnt, kC, g.ls);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const T x = sh[pos + k];
            dst[k] = (g0 + k < cnt) ? x : idle;
        }
        __syncthreads();
    };
    const T *dsrc = static_cast<const T *>(g.d) + base;
    const int ri = (int)(line * 2 * g.nch) + 2 * ch;  // this chunk's reduced rows
    T rx0 = T(0), rx1 = T(0);
    if (PASS == 1) {  // the chunk's end values from the reduced lines (block-uniform)
        rx0 = static_cast<const T *>(g.rx)[ri];
        rx1 = static_cast<const T *>(g.rx)[ri + 1];
    }
    if (g.mode == 0) {
        T va[kM], vb[kM], vc[kM], vd[kM];
        stage_load<T, kM>(va, static_cast<const T *>(g.a) + base, cnt);
        stage_load<T, kM>(vb, static_cast<const T *>(g.b) + base, cnt);
        stage_load<T, kM>(vc, static_cast<const T *>(g.c) + base, cnt);
        stage_load<T, kM>(vd, dsrc, cnt);
        asm volatile("" ::: "memory");  // keep the loads together, ahead of their uses
        put(va, ra, T(0));
        put(vb, rb, T(1));
        put(vc, rc, T(0));
        put(vd, rd, T(0));
    } else if (g.mode == 1) {
        T vs[kM], vd[kM], sv[kM];
        stage_load<T, kM>(vs, static_cast<const T *>(g.s) + base, cnt);
        stage_load<T, kM>(vd, dsrc, cnt);
        asm volatile("" ::: "memory");
        put(vs, sv, T(0));
        put(vd, rd, T(0));
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const bool v = g0 + k < cnt;
            ra[k] = v ? -sv[k] : T(0);
            rb[k] = T(1) + T(2) * sv[k];
            rc[k] = v ? -sv[k] : T(0);
        }
    } else {
        T vd[kM];
        stage_load<T, kM>(vd, dsrc, cnt);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            const bool v = g0 + k < cnt;
            ra[k] = v ? (T)g.ca : T(0);
            rb[k] = v ? (T)g.cb : T(1);
            rc[k] = v ? (T)g.cc : T(0);
        }
        put(vd, rd, T(0));
    }
    // the line's own ends: a at row 0 and c at row n-1 are not part of the system
    const i64 gl0 = (i64)ch * kC + g0;  // line row of this tile's first row
#pragma unroll
    for (int k = 0; k < kM; ++k) {
        if (gl0 + k == 0) ra[k] = T(0);
        if (gl0 + k == g.n - 1) rc[k] = T(0);
    }
    // the chunk's first and last rows (threads 0 and P-1), then identity rows there
    const bool first = p == 0, last = p == kP - 1;
    const T A0 = ra[0], B0 = rb[0], C0 = rc[0], D0 = rd[0];
    const T A1 = ra[kM - 1], B1 = rb[kM - 1], C1 = rc[kM - 1], D1 = rd[kM - 1];
    if (first) {
        ra[0] = T(0);
        rb[0] = T(1);
        rc[0] = T(0);
    }
    if (last) {
        ra[kM - 1] = T(0);
        rb[kM - 1] = T(1);
        rc[kM - 1] = T(0);
    }
    if (PASS == 0) {
        // one elimination, three right-hand sides: (0, d_1..d_{C-2}, 0), e_0 and
        // e_{C-1}.  The unit vectors only touch the chunk's identity end rows, so
        // their tile sweeps leave every interior dp zero: e_0 is the first row's
        // fd on tile 0, e_{C-1} the last row's ld on tile P-1.
        if (first) rd[0] = T(0);
        if (last) rd[kM - 1] = T(0);
        TileState<T, kM> ts;
        tile_eliminate<T, kM>(ra, rb, rc, rd, ts);
        const T ld3 = last ? T(1) : T(0);
        T f[3], lv[3];
        reduced_pcr3<T, kM>(ts, first ? T(1) : T(0), ld3, red, p, f, lv);
        T *RA = static_cast<T *>(g.ra), *RB = static_cast<T *>(g.rb);
        T *RC = static_cast<T *>(g.rc), *RD = static_cast<T *>(g.rd);
        // rows 1 and C-2 of the three solutions (interior rows of tiles 0 and P-1)
        const int k = first ? 1 : kM - 2;
        const T s1 = ts.dp[k] - ts.ap[k] * f[0] - ts.cp[k] * lv[0];
        const T s2 = -ts.ap[k] * f[1] - ts.cp[k] * lv[1];
        const T s3 = -ts.ap[k] * f[2] - ts.cp[k] * lv[2];
        if (first) {  // row 0: A0 u_prev + B0 u_0 + C0 u_1 = D0, u_1 = s1 + u_0 s2 + u_{C-1} s3
            RA[ri] = A0;
            RB[ri] = B0 + C0 * s2;
            RC[ri] = C0 * s3;
            RD[ri] = D0 - C0 * s1;
        }
        if (last) {  // row C-1 with u_{C-2} = s1 + u_0 s2 + u_{C-1} s3
            RA[ri + 1] = A1 * s2;
            RB[ri + 1] = B1 + A1 * s3;
            RC[ri + 1] = C1;
            RD[ri + 1] = D1 - A1 * s1;
        }
    } else {
        if (first) rd[0] = rx0;
        if (last) rd[kM - 1] = rx1;
        T u[kM];
        tile_solve<T, kM>(ra, rb, rc, rd, red, kP, kP, p, p, 1, u);
        __syncthreads();  // the reduced solve's last reads of the shared area are done
#pragma unroll
        for (int k = 0; k < kM; ++k) sh[pos + k] = u[k];
        __syncthreads();
        stage_out<T, kM>(static_cast<T *>(g.x) + base, sh, cnt, kC, g.ls);
    }
}

template <typename T>
hipError_t go(const ChunkArgs &g, i64 nlines, int pass, hipStream_t s) {
    const size_t shm = (size_t)std::max(g.ls, (pass == 0 ? 10 : 6) * kP) * sizeof(T);
    const i64 nb = nlines * g.nch;
    if (nb >= ((i64)1 << 31)) return hipErrorInvalidValue;
    if (pass == 0)
        launch(k_chunk<T, 0>, dim3((unsigned)nb), dim3(kP), shm, s, g);
    else
        launch(k_chunk<T, 1>, dim3((unsigned)nb), dim3(kP), shm, s, g);
    return hipGetLastError();
}

}  // namespace

i64 long_lines_chunks(i64 n) { return (n + kC - 1) / kC; }

size_t long_lines_workspace(const LineReq &r) {
    const size_t w = r.f64 ? 8 : 4;
    return 5 * (size_t)r.outer * 2 * (size_t)long_lines_chunks(r.n) * w + 5 * 256;
}

hipError_t launch_long_lines(const LineReq &r, void *ws, hipStream_t s, std::string *err) {
    const i64 nch = long_lines_chunks(r.n);
    if (r.inner != 1 || 2 * nch > 8192 || r.outer * 2 * nch >= ((i64)1 << 31)) {
        *err = "long lines must be contiguous and at most 8192 * 1024 rows";
        return hipErrorInvalidValue;
    }
    const size_t w = r.f64 ? 8 : 4;
    const size_t slot = ((size_t)r.outer * 2 * nch * w + 255) & ~(size_t)255;
    char *wb = static_cast<char *>(ws);
    ChunkArgs g;
    g.n = r.n;
    g.nch = (int)nch;
    g.ls = kP * (kM + 1);
    g.mode = r.mode == Mode::Arrays ? 0 : (r.mode == Mode::S ? 1 : 2);
    g.a = r.a;
    g.b = r.b;
    g.c = r.c;
    g.s = r.s;
    g.d = r.d;
    g.ca = r.ca;
    g.cb = r.cb;
    g.cc = r.cc;
    g.x = r.x;
    g.ra = wb;
    g.rb = wb + slot;
    g.rc = wb + 2 * slot;
    g.rd = wb + 3 * slot;
    g.rx = wb + 4 * slot;
    hipError_t e = r.f64 ? go<double>(g, r.outer, 0, s) : go<float>(g, r.outer, 0, s);
    if (e != hipSuccess) return e;
    // the reduced lines: 2 * nchunks rows each, coefficient arrays, one workgroup per line
    LineReq q;
    q.f64 = r.f64;
    q.mode = Mode::Arrays;
    q.out = Out::Store;
    q.a = g.ra;
    q.b = g.rb;
    q.c = g.rc;
    q.d = g.rd;
    q.x = wb + 4 * slot;
    q.inner = 1;
    q.n = 2 * nch;
    q.outer = r.outer;
    LinePlan pl;
    if (!plan_lines(q, &pl, err)) return hipErrorInvalidValue;
    e = launch_lines(q, pl, s);
    if (e != hipSuccess) return e;
    return r.f64 ? go<double>(g, r.outer, 1, s) : go<float>(g, r.outer, 1, s);
}

}  // namespace trid
