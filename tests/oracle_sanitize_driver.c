/* Test fixture: runs the FP64 oracle's table build and transport on inputs a test wrote to
 * files, in a process built with the host sanitizers (AddressSanitizer, UndefinedBehavior-
 * Sanitizer), and writes the outputs for the test to compare with the ordinary build.
 *
 * usage: driver <dir> <n_seg> <n_cols> <n_prm> <ne> <ns> <n_bins> <seed> <pid_end> <n_list>
 *   <dir>/segs.f64 [n_seg][n_cols], prm.f64 [n_prm], table.f64 (kind, theta_min, lo, hi),
 *   list_seg.u32 / list_pid.u32 [n_list]
 *   writes <dir>/counts.u64 [n_bins], counters.u64 [n_seg][7], records.f64 and list.f64 (REC
 *   doubles per particle, the oracle's record), theta.f64 [ne][ns], betamax.f64 [ne]
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define REC 9   /* the oracle's record: x, y, z, state, bin, events, diffusive steps, E, cos_in */

void or_build_table(int kind, double theta_min, int ne, int ns, double lo, double hi, double* theta,
                    double* betamax);
int or_run(const double* segs, int n_seg, const double* prm, const double* theta, const double* betamax,
           uint64_t seed, uint64_t pid_begin, uint64_t pid_end, int n_threads, uint64_t* counts,
           uint64_t* counters, double* records);
void or_run_list(const double* segs, int n_seg, const double* prm, const double* theta, const double* betamax,
                 uint64_t seed, const uint32_t* seg_ids, const uint32_t* pids, int64_t n, int n_threads,
                 double* records);

static void* load(const char* dir, const char* name, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(2);
    }
    void* p = malloc(bytes ? bytes : 1);
    if (bytes && fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read %s\n", path);
        exit(2);
    }
    fclose(f);
    return p;
}

static void save(const char* dir, const char* name, const void* p, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fclose(f);
}

int main(int argc, char** argv)
{
    if (argc != 11) {
        fprintf(stderr, "usage: %s dir n_seg n_cols n_prm ne ns n_bins seed pid_end n_list\n", argv[0]);
        return 2;
    }
    const char* dir = argv[1];
    const int n_seg = atoi(argv[2]), n_cols = atoi(argv[3]), n_prm = atoi(argv[4]);
    const int ne = atoi(argv[5]), ns = atoi(argv[6]);
    const size_t n_bins = (size_t)strtoull(argv[7], NULL, 10);
    const uint64_t seed = strtoull(argv[8], NULL, 10), pid_end = strtoull(argv[9], NULL, 10);
    const int64_t n_list = strtoll(argv[10], NULL, 10);

    double* segs = load(dir, "segs.f64", sizeof(double) * (size_t)n_seg * n_cols);
    double* prm = load(dir, "prm.f64", sizeof(double) * (size_t)n_prm);
    double* tab = load(dir, "table.f64", sizeof(double) * 4);
    double* theta = malloc(sizeof(double) * (size_t)ne * ns);
    double* betamax = malloc(sizeof(double) * (size_t)ne);
    or_build_table((int)tab[0], tab[1], ne, ns, tab[2], tab[3], theta, betamax);
    save(dir, "theta.f64", theta, sizeof(double) * (size_t)ne * ns);
    save(dir, "betamax.f64", betamax, sizeof(double) * (size_t)ne);

    uint64_t* counts = calloc(n_bins ? n_bins : 1, sizeof(uint64_t));
    uint64_t* counters = calloc((size_t)n_seg * 7, sizeof(uint64_t));
    /* one record per particle of [0, pid_end) of every segment (column 43: particles) */
    size_t n_rec = 0;
    for (int k = 0; k < n_seg; ++k) {
        const uint64_t N = (uint64_t)segs[(size_t)k * n_cols + 43];
        n_rec += N < pid_end ? N : pid_end;
    }
    double* records = calloc(n_rec ? n_rec * REC : 1, sizeof(double));
    or_run(segs, n_seg, prm, theta, betamax, seed, 0, pid_end, 2, counts, counters, records);
    save(dir, "counts.u64", counts, sizeof(uint64_t) * n_bins);
    save(dir, "counters.u64", counters, sizeof(uint64_t) * (size_t)n_seg * 7);
    save(dir, "records.f64", records, sizeof(double) * n_rec * REC);

    uint32_t* ls = load(dir, "list_seg.u32", sizeof(uint32_t) * (size_t)n_list);
    uint32_t* lp = load(dir, "list_pid.u32", sizeof(uint32_t) * (size_t)n_list);
    double* lrec = calloc(n_list ? (size_t)n_list * REC : 1, sizeof(double));
    or_run_list(segs, n_seg, prm, theta, betamax, seed, ls, lp, n_list, 2, lrec);
    save(dir, "list.f64", lrec, sizeof(double) * (size_t)n_list * REC);

    free(segs);
    free(prm);
    free(tab);
    free(theta);
    free(betamax);
    free(counts);
    free(counters);
    free(records);
    free(ls);
    free(lp);
    free(lrec);
    return 0;
}
