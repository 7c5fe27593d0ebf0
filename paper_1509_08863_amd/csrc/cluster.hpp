// Internal launchers of the normalisation and k-means kernels, for callers
// inside the library that run many independent problems in one launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace asc {

// count problems, problem b reads feature block b / fdiv (fstride elements
// apart) and owns centroids b (cstride), labels/distances b (lstride) and
// initial rows b (rows_stride).  The default is one problem.
// stamp (optional, count values): problem b is skipped by km_assign and
// km_update (its labels and centroids left as they are) while stamp[b] <
// want, and km_assign sets stamp[b] = mark (when mark != 0) if it changes a
// label of problem b.  With marks that only grow, a launch's blocks all see a
// problem the same way: a problem that runs can only be raised past want.
struct KmBatch {
    int count = 1;
    int64_t fstride = 0;
    int fdiv = 1;
    int64_t cstride = 0;
    int64_t lstride = 0;
    int64_t rows_stride = 0;
    uint32_t *stamp = nullptr;
    uint32_t want = 0;
    uint32_t mark = 0;
};

void km_normalize(float *Y, int64_t n, int64_t r, int64_t ldy, float *norms, hipStream_t s);
void km_init_rows(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *rows, int k, float *C,
                  const KmBatch &b, hipStream_t s);
// dist64 (optional): each row's squared distance to its centroid in float64
void km_assign(const float *F, int64_t n, int64_t r, int64_t ldf, const float *C, int k, int32_t *labels,
               float *dist2, double *dist64, const KmBatch &b, hipStream_t s);
size_t km_update_ws(int64_t n, int64_t r, int k, int count);
void km_update(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *labels, int k, float *C,
               int64_t *counts, void *ws, const KmBatch &b, hipStream_t s);
// stamp[0..count) = 0
void km_zero_stamps(uint32_t *stamp, int64_t count, hipStream_t s);
// b.count problems: C from the initial rows, iters Lloyd steps (assignment,
// update; ws: km_update_ws bytes) with each problem stopping at its fixed
// point, then an assignment that writes every row's float64 distance.
// stamp (b.count values) must hold less than base + 2 for every problem
// (zero, or an earlier call's stamps with a smaller base + iters + 1).
void km_lloyd(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *rows, int k, int iters, float *C,
              int32_t *labels, double *dist64, void *ws, uint32_t *stamp, uint32_t base, const KmBatch &b,
              hipStream_t s);
// groups x reps problems with labels and distances n apart: inert[g*reps + q]
// their inertias (fixed-order float64 sums), then per group the problem of
// least inertia (lowest on ties) copies its labels to lab_out[g*n] and, with
// C_out, its centroids (ckr floats, problems ckr apart) to C_out[g*ckr];
// inertia_out (optional) receives inert
void km_select(const double *dist64, const int32_t *lab_all, int64_t n, int groups, int reps, double *inert,
               int32_t *lab_out, double *inertia_out, const float *C_all, int64_t ckr, float *C_out, hipStream_t s);

}  // namespace asc
