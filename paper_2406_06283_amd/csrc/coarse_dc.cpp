// B_0^{-1} by divide and conquer over the block-tridiagonal structure of the coarse matrix.
//
// B_0 = Z^T B Z (eq. 2.23) couples the coarse vectors of two subdomains only when the subdomains
// overlap.  Let w be the largest index distance |i - j| of two coupled subdomains; grouping the
// subdomains into consecutive runs of w gives level blocks such that B_0 couples each level block
// only with its two neighbours: B_0 is block tridiagonal in them.  Its inverse is then built without
// a factorisation of the whole matrix:
//   * leaves: the inverse of every diagonal block (batched Gauss-Jordan with partial pivoting inside
//     the block, one launch; blocks beyond its size limit take an LU with partial pivoting and the two
//     triangular solves against P I);
//   * merges, level by level, of two adjacent ranges A (rows a, last level block l) and D (rows d,
//     first level block f), coupled only by U = B_0[l, f] and L = B_0[f, l]:
//       Q = L (A^-1)_ll U,   S = D - E_f Q E_f^T  (Schur complement of A),
//       S^-1 = D^-1 + D^-1 E_f (I - Q G)^-1 Q E_f^T D^-1,   G = (D^-1)_ff,
//       [A^-1 + X S_ff Y,  -X S^-1_(f,:) ;  -S^-1_(:,f) Y,  S^-1],  X = A^-1 E_l U,  Y = L E_l^T A^-1,
//     where the only inverse formed is that of the small matrix I - Q G (Gauss-Jordan or LU with
//     partial pivoting, as for the leaves).
// Every step is a batched launch over the merges of a level, so the serial chain is
// log2(#level blocks) small factorisations instead of one panel per 32 columns of B_0.  Pivoting
// stays inside the blocks: when any of the small factorisations meets a pivot that counts as zero,
// the caller falls back to the LU with partial pivoting of the whole (banded) B_0.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ctx.hpp"

namespace hkg {

namespace {

struct Range {
    int64_t r0, r1;       // coarse rows of the range
    int first, last;      // its first and last level block
};

// host-side job lists of one launch sequence, uploaded together
struct Blob {
    std::vector<uint8_t> bytes;
    template <typename T>
    size_t add(const std::vector<T> &v) {
        const size_t at = (bytes.size() + 255) / 256 * 256;
        bytes.resize(at + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(bytes.data() + at, v.data(), v.size() * sizeof(T));
        return at;
    }
};

}  // namespace

int32_t coarse_inverse_dc(hkgeneo_ctx *c, hipStream_t s, bool *done) {
    *done = false;
    const int ns = c->n_sub;
    const int64_t m0 = c->m0;
    const CoarsePairs &CP = c->CP;
    int wsub = 1;
    for (size_t t = 0; t < CP.pi.size(); ++t) {
        const int i = CP.pi[t], j = CP.pj[t];
        if (c->subs[i].m > 0 && c->subs[j].m > 0) wsub = std::max(wsub, std::abs(i - j));
    }
    // level blocks of wsub consecutive subdomains (empty ones dropped: two blocks with an empty one
    // between them are not coupled, which the merge formulas take as U = L = 0)
    std::vector<int64_t> b0v, b1v;
    int maxb = 0;
    for (int k0 = 0; k0 < ns; k0 += wsub) {
        const int k1 = std::min(k0 + wsub, ns);
        const int64_t a = c->subs[k0].offm, b = (k1 == ns) ? m0 : c->subs[k1].offm;
        if (b > a) {
            b0v.push_back(a);
            b1v.push_back(b);
            maxb = std::max(maxb, (int)(b - a));
        }
    }
    const int K = (int)b0v.size();
    if (K < 2 || maxb > 1024) return HKG_OK;

    // ---- plan ------------------------------------------------------------------------------------
    Blob blob;
    // leaves
    std::vector<DMat> leafLU(K), leafX(K);
    std::vector<int64_t> leafPoff(K);
    std::vector<TriJob> leafTri(K);
    std::vector<CopyJob> leafCopy(K), leafGJ(K);
    int64_t arenaLeaf = 0, pivLeaf = 0;
    for (int k = 0; k < K; ++k) {
        const int n = (int)(b1v[k] - b0v[k]);
        const int64_t d = b0v[k] + b0v[k] * m0;
        leafLU[k] = {arenaLeaf, n, n};
        leafX[k] = {d, n, (int32_t)m0};
        leafPoff[k] = pivLeaf;
        leafTri[k] = {arenaLeaf, d, n, n, n, (int32_t)m0};
        leafCopy[k] = {d, arenaLeaf, n, n, (int32_t)m0, n};
        leafGJ[k] = {d, d, n, n, (int32_t)m0, (int32_t)m0};
        arenaLeaf += (int64_t)n * n;
        pivLeaf += n;
    }
    // merge levels
    struct Level {
        int nm = 0, maxf = 0, maxa = 0, maxd = 0, maxl = 0;
        int64_t maxcopy = 0;
        size_t gTq, gQ, gW, gK, gPK, gUpd, gXa, gYa, gXaS, gAD, gDA, gAA;   // GemmJob sections
        size_t mW, mWinv, poff, tri, cp, gj;                               // DMat, poff, TriJob, CopyJob
    };
    std::vector<Level> levels;
    std::vector<Range> ranges(K);
    for (int k = 0; k < K; ++k) ranges[k] = {b0v[k], b1v[k], k, k};
    int64_t arenaMerge = 0, pivMerge = 0;
    int nflags = K;
    while (ranges.size() > 1) {
        Level L;
        std::vector<GemmJob> jTq, jQ, jW, jK, jPK, jUpd, jXa, jYa, jXaS, jAD, jDA, jAA;
        std::vector<DMat> mW, mWinv;
        std::vector<int64_t> poff;
        std::vector<TriJob> tri;
        std::vector<CopyJob> cp, gj;
        std::vector<Range> next;
        int64_t off = 0, poffv = 0;
        for (size_t q = 0; q + 1 < ranges.size(); q += 2) {
            const Range &A = ranges[q], &D = ranges[q + 1];
            const int64_t a0 = A.r0, l0 = b0v[A.last], d0 = D.r0, f0 = b0v[D.first];
            const int na = (int)(A.r1 - A.r0), nl = (int)(b1v[A.last] - l0), nd = (int)(D.r1 - D.r0),
                      nf = (int)(b1v[D.first] - f0);
            const int ld = (int)m0;
            const int64_t tq = off, qq = tq + (int64_t)nf * nl, w = qq + (int64_t)nf * nf, winv = w + (int64_t)nf * nf,
                          kk = winv + (int64_t)nf * nf, pm = kk + (int64_t)nf * nf, rm = pm + (int64_t)nd * nf,
                          pk = rm + (int64_t)nf * nd, xa = pk + (int64_t)nd * nf, ya = xa + (int64_t)na * nf,
                          xas = ya + (int64_t)nf * na;
            off = xas + (int64_t)na * nf;
            // GemmJob {offA, offB, offC, M, N, K, lda, ldb, ldc}
            jTq.push_back({f0 + l0 * m0, l0 + l0 * m0, tq, nf, nl, nl, ld, ld, nf});     // L (A^-1)_ll
            jQ.push_back({tq, l0 + f0 * m0, qq, nf, nf, nl, nf, ld, nf});               // Q = Tq U
            jW.push_back({qq, f0 + f0 * m0, w, nf, nf, nf, nf, ld, nf});                // W = I - Q G
            mW.push_back({w, nf, nf});
            mWinv.push_back({winv, nf, nf});
            poff.push_back(poffv);
            poffv += nf;
            tri.push_back({w, winv, nf, nf, nf, nf});
            gj.push_back({w, winv, nf, nf, nf, nf});
            jK.push_back({winv, qq, kk, nf, nf, nf, nf, nf, nf});                       // K = W^-1 Q
            cp.push_back({d0 + f0 * m0, pm, nd, nf, ld, nd});                           // D^-1 E_f
            cp.push_back({f0 + d0 * m0, rm, nf, nd, ld, nf});                           // E_f^T D^-1
            jPK.push_back({pm, kk, pk, nd, nf, nf, nd, nf, nd});                        // P K
            jUpd.push_back({pk, rm, d0 + d0 * m0, nd, nd, nf, nd, nf, ld});             // S^-1
            jXa.push_back({a0 + l0 * m0, l0 + f0 * m0, xa, na, nf, nl, ld, ld, na});    // X = A^-1 E_l U
            jYa.push_back({f0 + l0 * m0, l0 + a0 * m0, ya, nf, na, nl, ld, ld, nf});    // Y = L E_l^T A^-1
            jXaS.push_back({xa, f0 + f0 * m0, xas, na, nf, nf, na, ld, na});            // X S_ff
            jAD.push_back({xa, f0 + d0 * m0, a0 + d0 * m0, na, nd, nf, na, ld, ld});    // -X S^-1_(f,:)
            jDA.push_back({d0 + f0 * m0, ya, d0 + a0 * m0, nd, na, nf, ld, nf, ld});    // -S^-1_(:,f) Y
            jAA.push_back({xas, ya, a0 + a0 * m0, na, na, nf, na, nf, ld});             // A^-1 + X S_ff Y
            L.maxf = std::max(L.maxf, nf);
            L.maxa = std::max(L.maxa, na);
            L.maxd = std::max(L.maxd, nd);
            L.maxl = std::max(L.maxl, nl);
            L.maxcopy = std::max<int64_t>(L.maxcopy, (int64_t)nd * nf);
            next.push_back({A.r0, D.r1, A.first, D.last});
        }
        if (ranges.size() % 2) next.push_back(ranges.back());
        L.nm = (int)mW.size();
        L.gTq = blob.add(jTq);
        L.gQ = blob.add(jQ);
        L.gW = blob.add(jW);
        L.gK = blob.add(jK);
        L.gPK = blob.add(jPK);
        L.gUpd = blob.add(jUpd);
        L.gXa = blob.add(jXa);
        L.gYa = blob.add(jYa);
        L.gXaS = blob.add(jXaS);
        L.gAD = blob.add(jAD);
        L.gDA = blob.add(jDA);
        L.gAA = blob.add(jAA);
        L.mW = blob.add(mW);
        L.mWinv = blob.add(mWinv);
        L.poff = blob.add(poff);
        L.tri = blob.add(tri);
        L.cp = blob.add(cp);
        L.gj = blob.add(gj);
        arenaMerge = std::max(arenaMerge, off);
        pivMerge = std::max<int64_t>(pivMerge, poffv);
        nflags += L.nm;
        levels.push_back(L);
        ranges.swap(next);
    }
    const size_t sLeafLU = blob.add(leafLU), sLeafX = blob.add(leafX), sLeafPoff = blob.add(leafPoff),
                 sLeafTri = blob.add(leafTri), sLeafCopy = blob.add(leafCopy), sLeafGJ = blob.add(leafGJ);
    // every block every job touches lies inside its buffer (checked here, before any launch)
    const int64_t arena = std::max(arenaLeaf, arenaMerge), nX = m0 * m0;
    auto inside = [](int64_t off, int64_t rows, int64_t cols, int64_t ld, int64_t size) {
        return rows <= 0 || cols <= 0 || (off >= 0 && rows <= ld && off + (rows - 1) + (cols - 1) * ld < size);
    };
    {
        bool ok = true;
        for (int k = 0; k < K; ++k) {
            const int64_t n = leafLU[k].n;
            ok = ok && inside(leafLU[k].off, n, n, n, arena) && inside(leafX[k].off, n, n, m0, nX) &&
                 inside(leafCopy[k].offS, n, n, m0, nX);
        }
        for (const Level &L : levels) {
            struct Sec {
                size_t at;
                int64_t sa, sb, sc;
            };
            const Sec secs[] = {{L.gTq, nX, nX, arena},  {L.gQ, arena, nX, arena},   {L.gW, arena, nX, arena},
                                {L.gK, arena, arena, arena}, {L.gPK, arena, arena, arena}, {L.gUpd, arena, arena, nX},
                                {L.gXa, nX, nX, arena},   {L.gYa, nX, nX, arena},    {L.gXaS, arena, nX, arena},
                                {L.gAD, arena, nX, nX},   {L.gDA, nX, arena, nX},    {L.gAA, arena, arena, nX}};
            for (const Sec &q : secs)
                for (int t = 0; t < L.nm; ++t) {
                    const GemmJob &g = reinterpret_cast<const GemmJob *>(blob.bytes.data() + q.at)[t];
                    ok = ok && inside(g.offA, g.M, g.K, g.lda, q.sa) && inside(g.offB, g.K, g.N, g.ldb, q.sb) &&
                         inside(g.offC, g.M, g.N, g.ldc, q.sc);
                }
            const auto *cj = reinterpret_cast<const CopyJob *>(blob.bytes.data() + L.cp);
            for (int t = 0; t < 2 * L.nm; ++t)
                ok = ok && inside(cj[t].offS, cj[t].rows, cj[t].cols, cj[t].ldS, nX) &&
                     inside(cj[t].offD, cj[t].rows, cj[t].cols, cj[t].ldD, arena);
            const auto *gjj = reinterpret_cast<const CopyJob *>(blob.bytes.data() + L.gj);
            for (int t = 0; t < L.nm; ++t)
                ok = ok && inside(gjj[t].offS, gjj[t].rows, gjj[t].cols, gjj[t].ldS, arena) &&
                     inside(gjj[t].offD, gjj[t].rows, gjj[t].cols, gjj[t].ldD, arena);
        }
        if (!ok) {
            set_last_error("coarse divide and conquer: a block lies outside its buffer");
            return HKG_EINVAL;
        }
    }

    // ---- device buffers ----------------------------------------------------------------------------
    HKG_TRY(upload_staged(c, &c->wDCjobs, blob.bytes.data(), blob.bytes.size(), s));
    HKG_TRY(walloc(c, &c->wDC, (size_t)arena * sizeof(double)));
    HKG_TRY(walloc(c, &c->wDCpiv, (size_t)std::max(pivLeaf, pivMerge) * sizeof(int32_t)));
    HKG_TRY(walloc(c, &c->wDCinfo, (size_t)nflags * sizeof(int32_t)));
    if (c->B0inv.bytes != (size_t)(m0 * m0) * sizeof(double))
        HKG_TRY(dalloc(c, &c->B0inv, (size_t)(m0 * m0) * sizeof(double)));
    const uint8_t *jb = static_cast<const uint8_t *>(c->wDCjobs.p);
    auto J = [&](size_t at) { return reinterpret_cast<const GemmJob *>(jb + at); };
    double *ar = dp<double>(c->wDC), *X = dp<double>(c->B0inv);
    const double *B0 = dp<double>(c->wB0);
    int32_t *piv = dp<int32_t>(c->wDCpiv), *info = dp<int32_t>(c->wDCinfo);

    // ---- leaves: X[b, b] = B_0[b, b]^-1 ----------------------------------------------------------
    if (maxb <= inv_gj_max_n()) {
        HKG_TRY(inv_gj_batched(reinterpret_cast<const CopyJob *>(jb + sLeafGJ), K, maxb, B0, X, info, s));
    } else {
        HKG_TRY(copy_blocks_batched(reinterpret_cast<const CopyJob *>(jb + sLeafCopy), K, (int64_t)maxb * maxb, B0, ar,
                                    s));
        HKG_TRY(lu_batched<double>(reinterpret_cast<const DMat *>(jb + sLeafLU),
                                   reinterpret_cast<const int64_t *>(jb + sLeafPoff), K, maxb, ar, piv, info, true, s));
        HKG_TRY(perm_identity_batched<double>(reinterpret_cast<const DMat *>(jb + sLeafX),
                                              reinterpret_cast<const int64_t *>(jb + sLeafPoff), K, maxb, piv, X, s));
        const TriJob *lt = reinterpret_cast<const TriJob *>(jb + sLeafTri);
        HKG_TRY(tri_solve_batched<double>(lt, K, maxb, maxb, ar, X, TRI_LOWER_UNIT, s));
        HKG_TRY(tri_solve_batched<double>(lt, K, maxb, maxb, ar, X, TRI_UPPER, s));
    }

    // ---- merges ------------------------------------------------------------------------------------
    // Per level, the side stream computes X = A^-1 E_l U, Y = L E_l^T A^-1 and the copies of D^-1 E_f,
    // E_f^T D^-1 beside the chain that ends in the small inverse (they read only blocks that stay as
    // they are until S^-1 is formed), and later the two off-diagonal blocks beside X S_ff and the new
    // A block.  Every buffer region written on one stream is read on the other only after an event.
    hipStream_t s3 = c->s3;
    for (hipEvent_t &ev : c->ev_dc)
        if (!ev) HKG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    int flag0 = K;
    for (const Level &L : levels) {
        const int nm = L.nm, f = L.maxf;
        const DMat *mW = reinterpret_cast<const DMat *>(jb + L.mW);
        const int64_t *po = reinterpret_cast<const int64_t *>(jb + L.poff);
        const TriJob *tj = reinterpret_cast<const TriJob *>(jb + L.tri);
        HKG_HIP(hipEventRecord(c->ev_dc[0], s));
        HKG_HIP(hipStreamWaitEvent(s3, c->ev_dc[0], 0));
        HKG_TRY(gemm_batched<double>(J(L.gXa), nm, L.maxa, f, X, B0, ar, 1.0, 0.0, false, false, s3));
        HKG_TRY(gemm_batched<double>(J(L.gYa), nm, f, L.maxa, B0, X, ar, 1.0, 0.0, false, false, s3));
        HKG_TRY(copy_blocks_batched(reinterpret_cast<const CopyJob *>(jb + L.cp), 2 * nm, L.maxcopy, X, ar, s3));
        HKG_HIP(hipEventRecord(c->ev_dc[1], s3));
        HKG_TRY(gemm_batched<double>(J(L.gTq), nm, f, L.maxl, B0, X, ar, 1.0, 0.0, false, false, s));
        HKG_TRY(gemm_batched<double>(J(L.gQ), nm, f, f, ar, B0, ar, 1.0, 0.0, false, false, s));
        HKG_TRY(identity_batched(mW, nm, f, ar, s));
        HKG_TRY(gemm_batched<double>(J(L.gW), nm, f, f, ar, X, ar, -1.0, 1.0, false, false, s));
        if (f <= inv_gj_max_n()) {
            HKG_TRY(inv_gj_batched(reinterpret_cast<const CopyJob *>(jb + L.gj), nm, f, ar, ar, info + flag0, s));
        } else {
            HKG_TRY(lu_batched<double>(mW, po, nm, f, ar, piv, info + flag0, true, s));
            HKG_TRY(perm_identity_batched<double>(reinterpret_cast<const DMat *>(jb + L.mWinv), po, nm, f, piv, ar, s));
            HKG_TRY(tri_solve_batched<double>(tj, nm, f, f, ar, ar, TRI_LOWER_UNIT, s));
            HKG_TRY(tri_solve_batched<double>(tj, nm, f, f, ar, ar, TRI_UPPER, s));
        }
        HKG_TRY(gemm_batched<double>(J(L.gK), nm, f, f, ar, ar, ar, 1.0, 0.0, false, false, s));
        HKG_HIP(hipStreamWaitEvent(s, c->ev_dc[1], 0));
        HKG_TRY(gemm_batched<double>(J(L.gPK), nm, L.maxd, f, ar, ar, ar, 1.0, 0.0, false, false, s));
        HKG_TRY(gemm_batched<double>(J(L.gUpd), nm, L.maxd, L.maxd, ar, ar, X, 1.0, 1.0, false, false, s));
        HKG_HIP(hipEventRecord(c->ev_dc[2], s));
        HKG_HIP(hipStreamWaitEvent(s3, c->ev_dc[2], 0));
        HKG_TRY(gemm_batched<double>(J(L.gAD), nm, L.maxa, L.maxd, ar, X, X, -1.0, 0.0, false, false, s3));
        HKG_TRY(gemm_batched<double>(J(L.gDA), nm, L.maxd, L.maxa, X, ar, X, -1.0, 0.0, false, false, s3));
        HKG_HIP(hipEventRecord(c->ev_dc[3], s3));
        HKG_TRY(gemm_batched<double>(J(L.gXaS), nm, L.maxa, f, ar, X, ar, 1.0, 0.0, false, false, s));
        HKG_TRY(gemm_batched<double>(J(L.gAA), nm, L.maxa, L.maxa, ar, ar, X, 1.0, 1.0, false, false, s));
        HKG_HIP(hipStreamWaitEvent(s, c->ev_dc[3], 0));
        flag0 += nm;
    }
    std::vector<int32_t> flags(nflags);
    HKG_HIP(hipMemcpyAsync(flags.data(), info, nflags * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HKG_HIP(hipStreamSynchronize(s));
    for (int32_t v : flags)
        if (v) return HKG_OK;          // a block needs pivoting across blocks: the caller factors B_0 whole
    *done = true;
    return HKG_OK;
}

}  // namespace hkg
