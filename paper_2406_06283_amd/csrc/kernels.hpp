// Host-callable launch wrappers of the HIP kernels (all asynchronous on the given stream).
#pragma once

#include "internal.hpp"

namespace hkg {

enum { TRI_LOWER_UNIT = 0, TRI_UPPER = 1, TRI_LOWER_UNIT_TRANS = 2 };

// ---- dense.hip --------------------------------------------------------------------------------
template <typename T>
int32_t gemm_batched(const GemmJob *d_jobs, int nbatch, int maxM, int maxN, const T *A, const T *B, T *C, T alpha,
                     T beta, bool ta, bool tb, hipStream_t s);
template <typename T>
// P A = L U of every matrix (partial pivoting if `pivot`); band >= 0: the matrices are banded with that
// half-width, and the work is restricted to the band and the fill of the row exchanges
int32_t lu_batched(const DMat *d_mats, const int64_t *d_poff, int nbatch, int maxn, T *A, int32_t *piv,
                   int32_t *info, bool pivot, hipStream_t s, int band = -1);
template <typename T>
// band >= 0: op(T) has no entry farther than `band` from the diagonal.  Xin (banded lower solves
// with tri_band_fits only, square right-hand sides, T the packed L D L^T): Y = L^{-1} Xin^T (Xin
// with the layout of X) written as D^{-1/2} Y D^{-1/2} into X at the jobs' (offO, ldO); Xin untouched
int32_t tri_solve_batched(const TriJob *d_jobs, int nbatch, int maxn, int maxcol, const T *Tm, T *X, int mode,
                          hipStream_t s, int band = -1, const T *Xin = nullptr);
// whether the one-launch banded solve serves matrices of up to maxn rows with this half-bandwidth
bool tri_band_fits(int maxn, int band, size_t elem);
// Y = L^{-1} R for square right-hand sides, L the unit lower factor of the packed L D L^T Tm with
// half-bandwidth band: right-hand side c is row c of Xin at the jobs' (offX, ldX) (in_cols: its
// column c, with offX and ldX even); solution c is written as row c of Xout at (offO, ldO), with
// `scale` as D^{-1/2} Y D^{-1/2}.  Two combinations: (in rows, no scale), (in columns, scale).
bool tri_lower_window_fits(int maxn, int band);
int32_t tri_lower_window_batched(const TriJob *d_jobs, int nbatch, int maxn, int maxcol, const double *Tm,
                                 const double *Xin, bool in_cols, double *Xout, bool scale, int band,
                                 hipStream_t s);
// X = L^{-T} X in place for a few right-hand sides (the jobs' X at (offX, ldX)), L as above; fits as
// tri_lower_window_fits
int32_t tri_ltrans_window_batched(const TriJob *d_jobs, int nbatch, int maxn, int maxcol, const double *Tm, double *X,
                                  int band, hipStream_t s);
constexpr int LU_BLOCK = 32;    // block size of the dense LU, triangular solves and inversions

// diagonal LU_BLOCK blocks of L^{-1} (unit lower) and U^{-1} of one packed LU, into Linv / Uinv
int32_t tri_diag_inverse(const double *LU, int n, int ld, double *Linv, double *Uinv, int ldo, hipStream_t s);
// A^{-1} from a packed LU (P A = L U) by independent column solves in one launch, given the
// inverted LU_BLOCK diagonal blocks of L and U (tri_diag_inverse); needs lu_inverse_cols_lds(n)
// bytes of LDS per block; uband >= 0: U has no entry farther than uband above the diagonal
int64_t lu_inverse_cols_lds(int n);
int32_t lu_inverse_cols(const double *LU, int n, int ld, const int32_t *piv, const double *Linv, const double *Uinv,
                        int ldd, double *X, int ldx, int uband, hipStream_t s);
// out[:, c] = X[:, sigma(c)], P e_c = e_{sigma(c)} for the LU's row exchanges (so out = X P)
int32_t gather_pivot_columns(int n, const double *X, int ldx, const int32_t *piv, double *out, int ldo, hipStream_t s);
template <typename T>
int32_t perm_identity_batched(const DMat *d_mats, const int64_t *d_poff, int nbatch, int maxn, const int32_t *piv,
                              T *X, hipStream_t s);
template <typename T>
int32_t transpose_batched(const DMat *d_mats, int nbatch, int maxn, const T *in, T *out, hipStream_t s);
int32_t cast_f64_f32(const double *in, float *out, int64_t n, hipStream_t s);
// X = I for every matrix of the list
int32_t identity_batched(const DMat *d_mats, int nbatch, int maxn, double *X, hipStream_t s);
// Batched inverse by Gauss-Jordan with partial pivoting (one workgroup per matrix, the
// matrix in registers): out block = in block^{-1} for n <= inv_gj_max_n(); info[b] = 1 when a pivot
// is at most 32 n eps times the largest one or not finite.  Jobs: CopyJob {offS, offD, n, n, ldS, ldD}.
int inv_gj_max_n();
int32_t inv_gj_batched(const CopyJob *d_jobs, int nbatch, int maxn, const double *in, double *out, int32_t *info,
                       hipStream_t s);
// one rectangular block copy per job (src and dst must not overlap)
int32_t copy_blocks_batched(const CopyJob *d_jobs, int nbatch, int64_t max_elems, const double *src, double *dst,
                            hipStream_t s);

// ---- setup.hip: local blocks of every subdomain ---------------------------------------------------
struct SubDev {             // per-subdomain device descriptors
    int32_t nI, nG;
    int64_t offI, offG;     // into I_idx / G_idx and the concatenated local vectors
    int64_t offBIO;         // [B_II | B_IG], nI x (nI + nG), ld nI
    int64_t offSq;          // nI x nI work matrices (Schur, C_II, ...), ld nI
    int64_t offGG;          // nG x nG, ld nG
    int64_t offGI;          // nG x nI, ld nG
    int64_t offPiv;         // pivots (max(nI, nG))
    int32_t bandBeg, bandEnd;
    int64_t offZ;           // nI x m, ld nI
    int64_t offY;           // m x (nI + nG), ld m
    int32_t m, offm;        // eigenvectors kept, coarse offset
    int64_t offM;           // nI x nI, ld ldM: the local inverse B_D^{-1}, and the matrix tridiagonalised
    int32_t ldM, pad_;      // nI rounded up to 32 entries: every 64-row column segment starts on a line
};

int32_t form_operator(const double *A, const double *S, double k2, double *B, double *Dk, int64_t nnz, hipStream_t s);
int32_t extract_blocks(const SubDev *d_sub, int nsub, int maxnI, const int32_t *rowptr, const int32_t *colidx,
                       const double *Bval, const double *Dval, const int32_t *I_idx, const int32_t *G_idx,
                       const double *winv, double *BIO, double *CII, hipStream_t s);
int32_t assemble_gamma(const SubDev *d_sub, int nsub, int maxnG, int npe, const int32_t *band_elem,
                       const int32_t *band_loc, const double *elemK, const double *elemM, double k2, double *BGG,
                       hipStream_t s);
int32_t gather_gamma_rows(const SubDev *d_sub, int nsub, int maxnI, int maxnG, const double *BIO, double *GI,
                          hipStream_t s);
template <typename T>
int32_t apply_pivots_rows(const SubDev *d_sub, int nsub, int maxcol, const int32_t *piv, T *X, int which, hipStream_t s);
int32_t copy_bii(const SubDev *d_sub, int nsub, int maxnI, const double *BIO, double *out, hipStream_t s);
int32_t check_spd_pivots(const SubDev *d_sub, int nsub, const double *C, int32_t *flag, hipStream_t s);
// C_II = L D L^T in place (packed as an LU without exchanges) when its band fits the one-launch
// kernel (ldl_band_fits); C at offSq with ld n_I
bool ldl_band_fits(int maxnI, int band);
int32_t ldl_band(const SubDev *d_sub, int nsub, int maxnI, double *C, int band, hipStream_t s);
// T = D^{-1/2} S D^{-1/2} into the padded (offM, ldM) layout
int32_t scale_sym(const SubDev *d_sub, int nsub, int maxnI, const double *C, const double *S, double *T, hipStream_t s);

// ---- eigen.hip: tridiagonalisation, selection, eigenvectors --------------------------------------
int32_t tridiagonalize_blocked(const SubDev *d_sub, int nsub, int maxnI, double *Sq, double *VWV, double *d, double *e,
                               double *tau, hipStream_t s);
int32_t select_eigs(const SubDev *d_sub, int nsub, int maxnI, const double *d, const double *e, int mode, double tau,
                    int nev, double rtol, int mmax, int32_t *m_out, double *lam_out, int32_t *flag, double *iv,
                    hipStream_t s);
// inverse iteration for the selected eigenvectors of T (one wave per subdomain); max_nm = the
// largest n_I m_i (the iterates are staged in LDS when they fit)
int32_t tridiag_vectors_n(const SubDev *d_sub, int nsub, int maxnI, int64_t max_nm, const double *d, const double *e,
                          const double *lam, int mmax, double *Z, double *scratch, unsigned char *swp, hipStream_t s);
int32_t back_transform_n(const SubDev *d_sub, int nsub, int maxnI, int max_m, const double *Sq, const double *tau,
                         double *Z, hipStream_t s);
int32_t scale_rows_invsqrt_diag(const SubDev *d_sub, int nsub, const double *C, double *Z, hipStream_t s);
int32_t finish_basis(const SubDev *d_sub, int nsub, const int32_t *I_idx, const double *winv, double *Z,
                     hipStream_t s);
// Zr: the basis row-major (n_I x m_i at offZ); max_m: the largest m_i
int32_t coarse_pairs(int npairs, const int32_t *pi, const int32_t *pj, const int32_t *ptr, const int32_t *qi,
                     const int32_t *qj, const SubDev *d_sub, int max_m, const double *Y, const double *Zr, double *B0,
                     int m0, hipStream_t s);

// ---- apply.hip: one application of the two-level preconditioner ----------------------------------
struct ApplyPlan {
    int nsub, maxnI, nrhs, m0, two_level, local_f32, n_dof, max_m;
    const SubDev *d_sub;
    const int32_t *I_idx;
    const double *winv_loc;     // local prolongation weights per concatenated position (1 or 1/mu)
    const void *Minv;           // local inverses (float or double), nI x nI at offM, ld ldM
    const double *Z;            // Z_i column-major (n_I x m_i) at offZ
    const double *Zr;           // Z_i row-major (n_I x m_i) at offZ
    const double *B0inv;
    const int32_t *tp_ptr, *tp_pos, *tp_sub;
    double *u;                  // sum nI x nrhs
    double *c, *y;              // m0 x nrhs
    double *ypart;              // chunks x m0 x nrhs
    int64_t sum_nI;
    const int32_t *active = nullptr;           // optional per-rhs flags (FGMRES): skip inactive columns
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // optional: recorded around the local-solve kernel
    int accumulate = 0;                        // z += M^{-1} r instead of z = M^{-1} r
    // Minv == nullptr: the coarse correction alone (a coarse-only context of a nested decomposition)
};
int32_t apply_two_level(const ApplyPlan &p, const double *r, int ldr, double *z, int ldz, hipStream_t s);
int apply_ypart_chunks(int m0);
int32_t transpose_basis(const SubDev *d_sub, int nsub, const double *Z, double *Zr, hipStream_t s);

// coarse term of one position t of the transpose map (dof l in subdomain i at local index a): row a
// of Z_i in the row-major copy (zoff, m entries) and the slice y_i of the coarse vector (yoff)
struct TpCoarse {
    int64_t zoff;
    int32_t yoff, m;
};
int32_t tp_coarse(const SubDev *d_sub, const int32_t *tp_pos, const int32_t *tp_sub, int64_t ntp, TpCoarse *out,
                  hipStream_t s);

// ---- krylov.hip ------------------------------------------------------------------------------------
int32_t spmv(int n, int nrhs, const int32_t *rowptr, const int32_t *colidx, const double *val, const double *x,
             int ldx, double *y, int ldy, const double *f, int ldf, hipStream_t s, const int32_t *active = nullptr);

struct GmresDev {
    int n, nrhs, restart, nblk;
    double *V;          // n x (restart+1) per rhs, column stride n, rhs stride n*(restart+1)
    double *Zk;         // n x restart per rhs
    double *H;          // (restart+1) x restart per rhs, column-major
    double *cs, *sn;    // restart per rhs
    double *g;          // restart+1 per rhs
    double *part;       // nblk x (restart+2) partial sums per rhs
    double *hcol;       // restart+2 per rhs: current column before rotations
    double *scal;       // 8 per rhs: [beta0, fnorm, |g_{j+1}|, breakdown, ...]
    int32_t *active;    // per rhs
    int32_t *iters;     // per rhs: preconditioner applications so far
    int max_iter;
    // inner product of the Arnoldi process: the dot products read the columns of VD (V itself for
    // the Euclidean product; D_k V, stored in DV, for the D_k inner product, dk = 1)
    const double *VD = nullptr;
    double *DV = nullptr;
    int dk = 0;
};
// D_k-inner-product Arnoldi: DV[:, j+1] = D_k w for w = V[:, j+1] (j = -1: the cycle's first vector)
// with D_k = A + k2 S from the two CSR value arrays, and the partial sums of w . D_k w in the slot
// the Euclidean norm partials use; gmres_dk_reduce: out[rhs] = sqrt of their fixed-order sum
int32_t gmres_dk_norm(const GmresDev &G, int j, const int32_t *rowptr, const int32_t *colidx, const double *Aval,
                      const double *Sval, double k2, hipStream_t s);
int32_t gmres_dk_reduce(const GmresDev &G, double *out, hipStream_t s);
int32_t gmres_norm_init(const GmresDev &G, const double *r, int ldr, hipStream_t s);
int32_t gmres_arnoldi_step(const GmresDev &G, int j, hipStream_t s);
int32_t gmres_finish_cycle(const GmresDev &G, const int32_t *jd, double *x, int ldx, hipStream_t s);
int32_t vec_norms(int n, int nrhs, const double *x, int ldx, double *out, double *part, int nblk, hipStream_t s);

}  // namespace hkg
