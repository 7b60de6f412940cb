// Batched FGMRES over several set-up problems: descriptors shared by the host engine and the kernels
// of batch.hip.
//
// Every kernel takes the table of ProbDev descriptors and a flattened work list, so a single launch
// covers all (problem, subdomain or row block, right-hand side) items of the live set, whatever their
// sizes.  The Arnoldi index j and the state of each (problem, rhs) pair live on the device, so one
// iteration is the same launch sequence every time (captured once per index parity and replayed), and
// so is the restart phase that ends a pair's cycle, tests its true residual and starts the next
// cycle or retires it.  Pairs therefore restart independently, and problems can join or leave the
// live set at any iteration boundary.
#pragma once

#include "kernels.hpp"

namespace hkg {

constexpr int BROWS = 256;          // rows per row block (one per thread)
constexpr int LTILE = 128;          // rows of the local inverse per local-solve tile (two per lane)

// state of one (problem, rhs) pair, kept on the device
enum : int32_t {
    PS_DONE = 0,        // finished (or not started)
    PS_ITER = 1,        // inside an FGMRES cycle: the iteration kernels advance it
    PS_CYCLE_END = 2,   // cycle ended: the restart phase updates x and decides
    PS_NEW = 3,         // just admitted: the restart phase starts it from x = 0
    PS_START = 4,       // transient inside the restart phase
};

struct ProbDev {
    int32_t n, nsub, m0, maxnI, nblk, nrhs, restart, nchunk;
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
    const TpCoarse *tpc;                 // coarse term per transpose-map position (two-level only)
    // batch workspace of this problem
    double *u, *c, *ypart;                                   // apply (ypart holds y = B_0^{-1} c)
    double *V, *Zk, *H, *cs, *sn, *g, *part, *hcol, *scal;   // FGMRES, per rhs strides below
    int32_t *active, *iters;                                 // per rhs
    int32_t *jcur;                                           // two per rhs (parity double buffer)
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

// live: table indices of the g.nprob live problems (pair t of the per-pair kernels is
// (live[t / max_nrhs], t % max_nrhs)); work lists name table indices directly.
// mode 0: standalone application (xin -> xout); mode 1: FGMRES iteration (V[:, j] -> Zk[:, j])
// par: parity of the iteration (which half of the double-buffered Arnoldi index it reads)
// cblk: (problem, group of 4 coarse rows) blocks of the coarse product
int32_t batch_apply(const BatchGeom &g, const ProbDev *probs, const WorkItem *items, const WorkItem *rblk,
                    const WorkItem *cblk, int mode, int par, hipStream_t s, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
int32_t batch_arnoldi(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, int par, hipStream_t s);
// restart phase for PS_CYCLE_END / PS_NEW pairs: x update, true residual, stop or next cycle
int32_t batch_restart(const BatchGeom &g, const ProbDev *probs, const WorkItem *rblk, const int32_t *live,
                      hipStream_t s);

}  // namespace hkg
