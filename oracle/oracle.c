/*
 * CPU oracle for exact 256-bin byte histograms -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library.  It shares no code, header or table with the HIP path.
 *
 * What it computes: for b in 0..255, out[b] = number of i < n with in[i] == b.
 * The paper (Sec. III.A) treats each packed byte as a pixel value 0..255 and
 * asks for the exact histogram (Sec. I frames the problem as exact histogram
 * computation); this is that definition written out as a plain counting loop.
 * There is no blocking, vectorisation or reordering beyond what a reader can
 * check by eye.
 *
 * The timing helper runs the same plain loop on T threads, each over one
 * contiguous slice, and sums the per-thread partial histograms.  Summation of
 * integer counts is exact, so the result equals the one-thread loop.
 */
#define _POSIX_C_SOURCE 199309L
#include <pthread.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* out[b] += #{ i < n : in[i] == b } for b in 0..255 (accumulates). */
void oracle_hist_u8_acc(const uint8_t *in, size_t n, uint64_t *out)
{
    for (size_t i = 0; i < n; ++i)
        out[in[i]] += 1;
}

/* out[b] = #{ i < n : in[i] == b } (overwrites). */
void oracle_hist_u8(const uint8_t *in, size_t n, uint64_t *out)
{
    memset(out, 0, 256 * sizeof(uint64_t));
    oracle_hist_u8_acc(in, n, out);
}

/* Histograms of many buffers: out[j][b] for buffer j at offsets[j], sizes[j]. */
void oracle_hist_many(const uint8_t *base, const uint64_t *offsets, const uint64_t *sizes,
                      size_t count, uint64_t *out)
{
    for (size_t j = 0; j < count; ++j)
        oracle_hist_u8(base + offsets[j], (size_t)sizes[j], out + 256 * j);
}

struct slice_job {
    const uint8_t *in;
    size_t n;
    uint64_t part[256];
};

static void *slice_worker(void *arg)
{
    struct slice_job *job = (struct slice_job *)arg;
    oracle_hist_u8(job->in, job->n, job->part);
    return NULL;
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/*
 * Histogram of in[0..n) with `threads` threads, each over one contiguous slice.
 * Writes the summed histogram to out and returns the wall time in seconds, or
 * a negative value if a thread could not be started.
 */
double oracle_hist_timed(const uint8_t *in, size_t n, int threads, uint64_t *out)
{
    if (threads < 1)
        threads = 1;
    struct slice_job *jobs = (struct slice_job *)calloc((size_t)threads, sizeof(struct slice_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return -1.0;
    }
    size_t per = n / (size_t)threads;
    for (int t = 0; t < threads; ++t) {
        jobs[t].in = in + per * (size_t)t;
        jobs[t].n = (t == threads - 1) ? n - per * (size_t)t : per;
    }
    double t0 = now_s();
    int started = 0;
    int failed = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tids[t], NULL, slice_worker, &jobs[t]) != 0) {
            failed = 1;
            break;
        }
        started = t;
    }
    slice_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tids[t], NULL);
    double t1 = now_s();
    memset(out, 0, 256 * sizeof(uint64_t));
    for (int t = 0; t < threads; ++t)
        for (int b = 0; b < 256; ++b)
            out[b] += jobs[t].part[b];
    free(jobs);
    free(tids);
    return failed ? -1.0 : t1 - t0;
}
