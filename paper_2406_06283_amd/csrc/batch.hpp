// Batched FGMRES iteration over several set-up problems: descriptors shared by the host driver and
// the kernels of batch.hip.
//
// Every per-iteration kernel takes the table of ProbDev descriptors and a flattened work list, so a
// single launch covers all (problem, subdomain or row block, right-hand side) items of the batch,
// whatever their sizes.  The Arnoldi index j of each (problem, rhs) lives on the device (jcur) and is
// advanced by the last kernel of the iteration, so one iteration is the same launch sequence every
// time: it is captured once as a HIP graph and replayed.
#pragma once

#include "kernels.hpp"

namespace hkg {

constexpr int BROWS = 256;          // rows per row block (one per thread)

struct ProbDev {
    int32_t n, nsub, m0, maxnI, nchunk, nblk, nrhs, restart;
    int32_t local_f32, two_level, max_iter, ldu_pad;
    int64_t sum_nI;
    double rtol;
    // resident operators of the problem's context
    const int32_t *rowptr, *colidx;
    const double *Bval;
    const SubDev *subs;
    const int32_t *I_idx;
    const double *wloc;
    const void *Minv;
    const double *Z, *Zr, *B0inv;
    const int32_t *tp_ptr, *tp_pos;
    // batch workspace of this problem
    double *u, *c, *ypart;                                   // apply
    double *V, *Zk, *H, *cs, *sn, *g, *part, *hcol, *scal;   // FGMRES, per rhs strides below
    int32_t *active, *iters, *jcur;                          // per rhs
    double *rnorm;                                           // per rhs
    // vectors of the current call: apply input/output, solve right-hand sides and iterates
    const double *xin;
    double *xout;
    const double *f;
    double *x;
    int32_t ldin, ldout, ldf, ldx;
};

struct WorkItem {
    int32_t p, s;       // problem and subdomain / row block / coarse tile
};

// launch geometry of a batch (host side)
struct BatchGeom {
    int nprob = 0, max_nrhs = 0, max_tiles = 0, max_nI = 0;
    int nitems = 0, nrblk = 0, ncblk = 0, restart = 0;
    bool any_coarse = false;
    int local_waves = 8;        // chosen by the autotuner
};

// mode 0: standalone application (xin -> xout); mode 1: FGMRES iteration (V[:, j] -> Zk[:, j])
int32_t batch_apply(const BatchGeom &g, const ProbDev *probs, const WorkItem *items, const WorkItem *rblk,
                    const WorkItem *cblk, int mode, hipStream_t s, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
int32_t batch_arnoldi(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, hipStream_t s);
// residual r = f - B x into V[:, 0] and its norm into rnorm (x = 0: the norm of f into scal[1] too)
int32_t batch_residual(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, int init, hipStream_t s);
int32_t batch_cycle_start(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, const int32_t *want,
                          hipStream_t s);
int32_t batch_cycle_update(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, hipStream_t s);

}  // namespace hkg
