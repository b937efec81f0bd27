/*
 * Plain CPU oracle for per-event pixel clustering.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file: only the tests, the smoke check and the benchmark's CPU-baseline leg
 * use it.  It shares no code, header or constant table with the device library.
 *
 * What it computes.  The paper names the work the offload pattern hands to the
 * co-processor only by its role: a "ClusterProducer" that turns the raw detector
 * data into clusters, which hits are then made from (Figure 1, Sec. 3; the
 * co-processor variant goes from raw data to hits directly).  The definition
 * written out below is the textbook one:
 *
 *   1. digis are fired pixels (module, row, col, adc), grouped by ascending module;
 *      module < n_modules, row < 160, col < 416, no pixel fired twice;
 *   2. two digis are connected iff they are in the same module and their rows and
 *      their columns each differ by at most one (8-connectivity, no wrap-around);
 *   3. a cluster is a connected component; its id is the smallest linear pixel
 *      index  module*66560 + col*160 + row  of its members, its charge is the sum
 *      of their adc (uint32 arithmetic) and its size the number of members;
 *   4. a cluster is kept iff charge >= charge_cut;
 *   5. outputs: kept clusters sorted by ascending id; per digi the id of its
 *      cluster if kept, else -1; the number of kept clusters.
 *   6. hits (the product the figure derives from clusters): per kept cluster its
 *      charge-weighted centroid in pixel units, x = sum(adc*col)/charge and
 *      y = sum(adc*row)/charge, from exact 64-bit sums divided in double precision
 *      and rounded to float; NaN for a cluster of zero charge.
 *
 * Components are found by breadth-first search over a dense 160x416 grid of digi
 * indices, one module at a time: slow, single-threaded and easy to check.
 *
 * Errors (checked in this order; the first class found is reported):
 *   out-of-range module/row/col -> -6, module ids decreasing -> -7,
 *   the same pixel fired twice  -> -5.  Outputs are unspecified on error.
 *
 * Digis in any order (pxo_cluster_event_any_order): the raw data of the figure's
 * producer carries no grouping, and the definition above does not depend on the
 * order of the digis.  That entry point first groups the digis by module with a
 * stable counting sort (count per module, exclusive prefix, place in input order),
 * runs the grouped definition on the grouped copy and returns every per-digi id at
 * the digi's input position.  No order error exists there: out of range -> -6, the
 * same pixel fired twice -> -5.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_ROWS 160
#define O_COLS 416

#define O_OK 0
#define O_E_INVAL (-1)
#define O_E_DUP (-5)
#define O_E_RANGE (-6)
#define O_E_ORDER (-7)
#define O_E_NOMEM (-9)

typedef struct {
    int64_t id;
    uint32_t charge;
    uint32_t size;
    uint64_t sum_col;   /* sum of adc*col */
    uint64_t sum_row;   /* sum of adc*row */
} o_cluster;

static int cmp_cluster(const void* a, const void* b)
{
    int64_t x = ((const o_cluster*)a)->id, y = ((const o_cluster*)b)->id;
    return (x > y) - (x < y);
}

/* Returns 0 on success or a negative error code; err_bits gets 1 (range), 2 (order),
 * 4 (duplicate pixel) for every class detected. */
/* As pxo_cluster_event, and per kept cluster its hit (hit_x, hit_y may be NULL). */
int pxo_cluster_event_hits(const uint16_t* module, const uint16_t* row, const uint16_t* col,
                           const uint16_t* adc, uint32_t n, uint32_t n_modules,
                           uint32_t charge_cut, int32_t* digi_cluster, int32_t* cl_id,
                           int32_t* cl_charge, int32_t* cl_size, uint32_t* n_clusters,
                           uint32_t* err_bits, float* hit_x, float* hit_y)
{
    uint32_t bits = 0;
    *n_clusters = 0;
    if (n > 0 && (!module || !row || !col || !adc || !digi_cluster))
        return O_E_INVAL;

    /* 1. range and order checks over every digi */
    for (uint32_t i = 0; i < n; ++i) {
        if (module[i] >= n_modules || row[i] >= O_ROWS || col[i] >= O_COLS)
            bits |= 1u;
        if (i > 0 && module[i] < module[i - 1])
            bits |= 2u;
    }
    if (bits) {
        if (err_bits) *err_bits = bits;
        return (bits & 1u) ? O_E_RANGE : O_E_ORDER;
    }

    int32_t* grid = (int32_t*)malloc(sizeof(int32_t) * O_ROWS * O_COLS);
    int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * (n ? n : 1));   /* component of digi */
    uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    o_cluster* cls = (o_cluster*)malloc(sizeof(o_cluster) * (n ? n : 1));
    if (!grid || !comp || !queue || !cls) {
        free(grid); free(comp); free(queue); free(cls);
        return O_E_NOMEM;
    }
    for (int k = 0; k < O_ROWS * O_COLS; ++k) grid[k] = -1;
    uint32_t n_comp = 0;

    uint32_t s = 0;
    while (s < n) {
        /* 2. the digis of one module: [s, e) */
        uint32_t e = s;
        while (e < n && module[e] == module[s]) ++e;
        for (uint32_t i = s; i < e; ++i) {
            int32_t* cell = &grid[row[i] * O_COLS + col[i]];
            if (*cell != -1) bits |= 4u;
            else *cell = (int32_t)i;
            comp[i] = -1;
        }
        /* 3. breadth-first search from every digi not yet reached */
        for (uint32_t i = s; i < e; ++i) {
            if (comp[i] != -1) continue;
            if (grid[row[i] * O_COLS + col[i]] != (int32_t)i) {  /* duplicate of another */
                comp[i] = -2;
                continue;
            }
            uint32_t head = 0, tail = 0;
            queue[tail++] = i;
            comp[i] = (int32_t)n_comp;
            int64_t min_lin = INT64_MAX;
            uint32_t charge = 0, size = 0;
            uint64_t sum_col = 0, sum_row = 0;
            while (head < tail) {
                uint32_t d = queue[head++];
                int64_t lin = (int64_t)module[d] * (O_ROWS * O_COLS) + (int64_t)col[d] * O_ROWS + row[d];
                if (lin < min_lin) min_lin = lin;
                charge += adc[d];
                size += 1;
                sum_col += (uint64_t)adc[d] * col[d];
                sum_row += (uint64_t)adc[d] * row[d];
                for (int dr = -1; dr <= 1; ++dr) {
                    for (int dc = -1; dc <= 1; ++dc) {
                        int r2 = (int)row[d] + dr, c2 = (int)col[d] + dc;
                        if ((dr == 0 && dc == 0) || r2 < 0 || r2 >= O_ROWS || c2 < 0 || c2 >= O_COLS)
                            continue;
                        int32_t nb = grid[r2 * O_COLS + c2];
                        if (nb >= 0 && comp[nb] == -1) {
                            comp[nb] = (int32_t)n_comp;
                            queue[tail++] = (uint32_t)nb;
                        }
                    }
                }
            }
            cls[n_comp].id = min_lin;
            cls[n_comp].charge = charge;
            cls[n_comp].size = size;
            cls[n_comp].sum_col = sum_col;
            cls[n_comp].sum_row = sum_row;
            ++n_comp;
        }
        /* reset the grid cells this module used */
        for (uint32_t i = s; i < e; ++i) grid[row[i] * O_COLS + col[i]] = -1;
        s = e;
    }

    if (bits) {
        free(grid); free(comp); free(queue); free(cls);
        if (err_bits) *err_bits = bits;
        return O_E_DUP;
    }

    /* 4./5. cut, per-digi ids, clusters in ascending id order */
    for (uint32_t i = 0; i < n; ++i) {
        const o_cluster* c = &cls[comp[i]];
        digi_cluster[i] = (c->charge >= charge_cut) ? (int32_t)c->id : -1;
    }
    qsort(cls, n_comp, sizeof(o_cluster), cmp_cluster);
    uint32_t k = 0;
    for (uint32_t j = 0; j < n_comp; ++j) {
        if (cls[j].charge < charge_cut) continue;
        if (cl_id) cl_id[k] = (int32_t)cls[j].id;
        if (cl_charge) cl_charge[k] = (int32_t)cls[j].charge;
        if (cl_size) cl_size[k] = (int32_t)cls[j].size;
        if (hit_x) hit_x[k] = cls[j].charge ? (float)((double)cls[j].sum_col / (double)cls[j].charge) : NAN;
        if (hit_y) hit_y[k] = cls[j].charge ? (float)((double)cls[j].sum_row / (double)cls[j].charge) : NAN;
        ++k;
    }
    *n_clusters = k;
    if (err_bits) *err_bits = 0;
    free(grid); free(comp); free(queue); free(cls);
    return O_OK;
}

int pxo_cluster_event(const uint16_t* module, const uint16_t* row, const uint16_t* col,
                      const uint16_t* adc, uint32_t n, uint32_t n_modules,
                      uint32_t charge_cut, int32_t* digi_cluster, int32_t* cl_id,
                      int32_t* cl_charge, int32_t* cl_size, uint32_t* n_clusters,
                      uint32_t* err_bits)
{
    return pxo_cluster_event_hits(module, row, col, adc, n, n_modules, charge_cut, digi_cluster, cl_id,
                                  cl_charge, cl_size, n_clusters, err_bits, NULL, NULL);
}

/* All clusters before the cut, sorted by id (for invariant tests): returns the count. */
int64_t pxo_components(const uint16_t* module, const uint16_t* row, const uint16_t* col,
                       const uint16_t* adc, uint32_t n, uint32_t n_modules,
                       int32_t* digi_cluster, int32_t* cl_id, int32_t* cl_charge,
                       int32_t* cl_size)
{
    uint32_t nc = 0, bits = 0;
    int rc = pxo_cluster_event(module, row, col, adc, n, n_modules, 0u, digi_cluster, cl_id,
                               cl_charge, cl_size, &nc, &bits);
    return rc == O_OK ? (int64_t)nc : (int64_t)rc;
}

/* Digis in any order: group by module (stable counting sort), cluster the grouped
 * copy with the definition above, per-digi ids back at the input positions. */
int pxo_cluster_event_any_order(const uint16_t* module, const uint16_t* row, const uint16_t* col,
                                const uint16_t* adc, uint32_t n, uint32_t n_modules,
                                uint32_t charge_cut, int32_t* digi_cluster, int32_t* cl_id,
                                int32_t* cl_charge, int32_t* cl_size, uint32_t* n_clusters,
                                uint32_t* err_bits, float* hit_x, float* hit_y)
{
    *n_clusters = 0;
    if (n > 0 && (!module || !row || !col || !adc || !digi_cluster))
        return O_E_INVAL;
    uint32_t bits = 0;
    for (uint32_t i = 0; i < n; ++i)
        if (module[i] >= n_modules || row[i] >= O_ROWS || col[i] >= O_COLS)
            bits |= 1u;
    if (bits) {
        if (err_bits) *err_bits = bits;
        return O_E_RANGE;
    }
    uint32_t* start = (uint32_t*)calloc((size_t)n_modules + 1, sizeof(uint32_t));
    uint32_t* pos = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));      /* grouped slot -> input index */
    uint16_t* g = (uint16_t*)malloc(sizeof(uint16_t) * 4 * (n ? n : 1));
    int32_t* gd = (int32_t*)malloc(sizeof(int32_t) * (n ? n : 1));
    if (!start || !pos || !g || !gd) {
        free(start); free(pos); free(g); free(gd);
        return O_E_NOMEM;
    }
    /* count per module, exclusive prefix, then every digi in input order to the next
     * free slot of its module */
    for (uint32_t i = 0; i < n; ++i) start[module[i] + 1] += 1;
    for (uint32_t m = 0; m < n_modules; ++m) start[m + 1] += start[m];
    for (uint32_t i = 0; i < n; ++i) pos[start[module[i]]++] = i;
    uint16_t *gm = g, *gr = g + n, *gc = g + 2 * (size_t)n, *ga = g + 3 * (size_t)n;
    for (uint32_t j = 0; j < n; ++j) {
        gm[j] = module[pos[j]];
        gr[j] = row[pos[j]];
        gc[j] = col[pos[j]];
        ga[j] = adc[pos[j]];
    }
    int rc = pxo_cluster_event_hits(gm, gr, gc, ga, n, n_modules, charge_cut, gd, cl_id, cl_charge, cl_size,
                                    n_clusters, err_bits, hit_x, hit_y);
    if (rc == O_OK)
        for (uint32_t j = 0; j < n; ++j) digi_cluster[pos[j]] = gd[j];
    free(start); free(pos); free(g); free(gd);
    return rc;
}
