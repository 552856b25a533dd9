// Built-in tuning table of libpbit (included once, by pbit_capi.hip).
// Entries: {kind (0 one list, 1 many lists), key bits M, largest node count
// n_max, pattern bits K, short-list cutoff}.  Written by
// paper_cs_0511020_amd/tune.py from device measurements (tuning.json beside
// the package holds the timings).
static const TuneEntry kBuiltinTuning[] = {
    {0, 8, 0xFFFFFFFFull, 8, 4096},
    {0, 16, 0xFFFFFFFFull, 8, 4096},
    {0, 32, 0xFFFFFFFFull, 8, 4096},
    {0, 64, 0xFFFFFFFFull, 8, 4096},
    {1, 8, 0x3930FEull, 8, 4096},
    {1, 8, 0x2CEDF90ull, 8, 1024},
    {1, 8, 0xFFFFFFFFull, 8, 2048},
    {1, 16, 0xFFFFFFFFull, 8, 2048},
    {1, 32, 0x407661ull, 8, 4096},
    {1, 32, 0xFFFFFFFFull, 8, 2048},
    {1, 64, 0xFFFFFFFFull, 8, 2048},
};
