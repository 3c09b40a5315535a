// Launchers of the step kernels (defined in kernels.hip).
#pragma once
#include "sol_dev.hpp"

namespace sol {

// Process-wide count of the device work items the library has queued:
// kernel dispatches (graph nodes included) and device copies.  Every kernel
// launch of the library goes through SOL_LAUNCH.
void note_dispatch(long n);
long dispatch_count();
#define SOL_LAUNCH(...)                \
    do {                               \
        ::sol::note_dispatch(1);       \
        hipLaunchKernelGGL(__VA_ARGS__); \
    } while (0)

void launch_asm_const(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s);
// fwd: the forward (residual-probing) assembly kernels instead of the
// stencil kernels (same systems, up to rounding)
void launch_asm_momentum(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s, int fwd = 0);
void launch_asm_transport(int dim, const CaseDev *c, const Tile *t, int nt, int vel_src, hipStream_t s, int fwd = 0);
void launch_div_rhs(int dim, const CaseDev *c, const Tile *t, int nt, int vel_src, hipStream_t s);
void launch_case_mean(const CaseDev *c, const int32_t *cidx, int ncase, hipStream_t s);
void launch_sub_mean(const CaseDev *c, const Tile *t, int nt, hipStream_t s);
void launch_project(const CaseDev *c, const Tile *t, int nt, hipStream_t s);
void launch_phase_commit(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s);

// two: BiCGSTAB preconditioned by two Jacobi sweeps instead of one; s1: the
// one-sweep 7-point solves of the launch all go through LDS (KJob::staged)
void launch_kinit(int kind, int nd, int fp32, bool two, bool s1, const KJob *j, const JTile *t, int nt, int k,
                  int mode, size_t smem, hipStream_t s);
void launch_kfinish(int nd, const KJob *j, const JTile *t, int nt, hipStream_t s);
void launch_kdecide(const KJob *j, int njobs, hipStream_t s);
// iteration kernels, all with the signature (jobs, tiles, const int *kbase,
// int koff): iteration index = (kbase ? *kbase : 0) + koff
enum KIter {
    KI_CG = 0, KI_BICG_A = 1, KI_BICG_B = 2,
    KI_MG_PQ = 4, KI_MG_DOWN0 = 5, KI_MG_DOWN = 6, KI_MG_EXACT = 7, KI_MG_UP = 8, KI_MG_UP0 = 9,
    KI_MG_DOWN0_INIT = 10,
    KI_MG_DOWN2 = 11, KI_MG_UP2 = 12       // two coarse levels in one launch
};
// kernel address of an iteration kernel (direct launches and graph nodes);
// two selects the two-sweep BiCGSTAB kernels, s1 the staged one-sweep ones
const void *kiter_fn(int which, int nd, int fp32, bool two, bool s1);
const void *mg_fn(int which, int nd, int fp32);
// workgroups of a fused pair of coarse levels (l, l+1); M = level l+1
int mg_fused_bricks(int dim, const MLevel &M);
// multigrid: start of the solves (r = b - A x, p = 0, partial (b, b)) and
// the inverse diagonal of level l >= 1 (FP32 copy when mi32 is given)
void launch_mg_init(int nd, int fp32, const KJob *j, const JTile *t, int nt, int k, int mode, hipStream_t s);
void launch_mg_finish(int nd, const KJob *j, const JTile *t, int nt, hipStream_t s);
void launch_mg_ir_resid(int nd, const KJob *j, const JTile *t, int nt, int mode, hipStream_t s);
void launch_mg_minv(int dim, const MLevel *lev, int l, int n, double *mi, float *mi32, hipStream_t s);
// multigrid: dense inverse of the exactly solved level l (n cells; work:
// 4 n + 1 doubles of device scratch)
void launch_mg_pinv(int dim, const MLevel *lev, int l, int n, double *P, float *P32, double *work, hipStream_t s);
const void *kbase_add_fn();   // (int *kbase, int m)
void launch_kbase_set(int *kbase, int v, hipStream_t s);
void launch_tune_rhs(void *b, int fp32, int n, hipStream_t s);
void launch_ir_resid(int nd, const KJob *j, const JTile *t, int nt, int mode, hipStream_t s);
void launch_ir_decide(const KJob *j, int njobs, int mode, int max_outer, hipStream_t s);
void launch_ir_update(int nd, const KJob *j, const JTile *t, int nt, hipStream_t s);
void launch_ir_close(const KJob *j, int njobs, hipStream_t s);
void launch_case_stats(const CaseDev *c, const int32_t *cidx, int ncase, hipStream_t s);
// initial guesses of the pressure-correction and energy solves; history reset
void launch_guess(const CaseDev *c, const Tile *t, int nt, hipStream_t s);
void launch_guess_mom(const CaseDev *c, const Tile *t, int nt, hipStream_t s);
void launch_hist_reset(const CaseDev *c, int ncase, hipStream_t s);

void launch_csr(int dim, const CaseDev *cd, int s, int n, int32_t *cnt, int32_t *row_ptr, int32_t *col,
                double *val, int build_pattern, hipStream_t st);
// the CSR export in two parts: row counts and their exclusive scan (cnt: n
// ints, row_ptr: n + 1), then the columns and values of rows [r0, r1) into
// arrays that start at entry `base` of the system's CSR arrays
void launch_csr_pattern(int dim, const CaseDev *cd, int s, int n, int32_t *cnt, int32_t *row_ptr, hipStream_t st);
void launch_csr_rows(int dim, const CaseDev *cd, int s, int r0, int r1, const int32_t *row_ptr, int base,
                     int32_t *col, double *val, hipStream_t st);
void launch_fill(double *x, double v, int n, hipStream_t s);
void launch_set_status(KState *st, int n, int status, hipStream_t s);

}  // namespace sol
