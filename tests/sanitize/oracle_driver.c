/*
 * Test driver that runs the oracle (oracle/transport.c, compiled into this
 * translation unit) as a standalone program, so that it can be built with
 * the CPU sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer, or
 * ThreadSanitizer for its pthread pool) without loading a sanitized library
 * into Python.
 *
 * Input file (little-endian, written by tests/test_oracle_sanitizers.py):
 *   int32 n_slabs, n_materials, msc, n_threads
 *   double half_width, B[3], ecut
 *   uint64 seed, n_prim, n_states
 *   uint32 n_rows, pad
 *   double z_planes[n_slabs + 1]; int32 slab_material[n_slabs]
 *   double tables[n_materials * 8 * 181]; double x0_cm[n_materials]
 *   orc_track prims[n_prim]; uint32 rows[n_prim]
 *   orc_track states[n_states]          (single steps of given states)
 * Output file:
 *   uint64 steps; double edep[n_rows * n_slabs]; orc_ledger ledger[n_rows]
 *   orc_track states_after[n_states]; orc_step_result results[n_states]
 */
#include <stdio.h>

#include "../../oracle/transport.c"

static void* read_all(FILE* f, size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (bytes && fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[4];
    double geo[5];
    uint64_t counts[3];
    uint32_t rows_pad[2];
    if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(geo, sizeof geo, 1, f) != 1 ||
        fread(counts, sizeof counts, 1, f) != 1 || fread(rows_pad, sizeof rows_pad, 1, f) != 1)
        return 2;
    const int n_slabs = hdr[0], n_mat = hdr[1];
    const uint64_t n_prim = counts[1], n_states = counts[2];
    const uint32_t n_rows = rows_pad[0];
    double* zp = (double*)read_all(f, sizeof(double) * (size_t)(n_slabs + 1));
    int32_t* sm = (int32_t*)read_all(f, sizeof(int32_t) * (size_t)n_slabs);
    double* tab = (double*)read_all(f, sizeof(double) * (size_t)n_mat * ORC_NTAB * ORC_NNODES);
    double* x0 = (double*)read_all(f, sizeof(double) * (size_t)n_mat);
    orc_track* prims = (orc_track*)read_all(f, sizeof(orc_track) * n_prim);
    uint32_t* rows = (uint32_t*)read_all(f, sizeof(uint32_t) * n_prim);
    orc_track* states = (orc_track*)read_all(f, sizeof(orc_track) * n_states);
    fclose(f);

    orc_problem pb;
    memset(&pb, 0, sizeof pb);
    pb.n_slabs = n_slabs;
    pb.n_materials = n_mat;
    pb.z_planes = zp;
    pb.slab_material = sm;
    pb.half_width = geo[0];
    pb.B[0] = geo[1];
    pb.B[1] = geo[2];
    pb.B[2] = geo[3];
    pb.tables = tab;
    pb.ecut = geo[4];
    pb.seed = counts[0];
    pb.msc = hdr[2];
    pb.x0_cm = x0;

    double* edep = (double*)malloc(sizeof(double) * (size_t)n_rows * (size_t)n_slabs);
    orc_ledger* led = (orc_ledger*)malloc(sizeof(orc_ledger) * n_rows);
    uint64_t steps = orc_run_events(&pb, prims, rows, n_prim, n_rows, edep, led, hdr[3]);
    orc_step_result* res = (orc_step_result*)calloc(n_states ? n_states : 1, sizeof(orc_step_result));
    for (uint64_t i = 0; i < n_states; ++i) orc_step(&pb, &states[i], &res[i]);

    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(&steps, sizeof steps, 1, o);
    fwrite(edep, sizeof(double), (size_t)n_rows * (size_t)n_slabs, o);
    fwrite(led, sizeof(orc_ledger), n_rows, o);
    fwrite(states, sizeof(orc_track), n_states, o);
    fwrite(res, sizeof(orc_step_result), n_states, o);
    fclose(o);
    free(zp); free(sm); free(tab); free(x0); free(prims); free(rows); free(states);
    free(edep); free(led); free(res);
    return 0;
}
