// host_checks.cpp -- the library's host code (argument validation, work
// planning, launch layout, sorting, the autotune cache and the C ABI's error
// paths) built without device code and run under AddressSanitizer and
// UndefinedBehaviorSanitizer on the CPU.  Test infrastructure: built and run
// by tests/test_sanitizers.py.
//
// The host library is compiled in this translation unit (#include of its
// source) so that its internal functions can be called directly; the device
// launchers it links against are replaced by stubs that report "not
// supported", and no check here reaches one of them.

#include "pms_api.hip"

#include <cassert>
#include <cstdio>
#include <random>
#include <set>

namespace pms {
hipError_t launch_windows(const pms_win_job*, int32_t, int32_t, const uint8_t*, uint32_t*,
                          uint32_t*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_search(const pms_dev_instance*, const pms_work_item*, uint32_t, pms_dev_state*,
                         pms_dev_counters*, uint32_t, uint32_t, uint32_t, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_fill(uint32_t*, uint64_t, uint32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_gather(const uint32_t*, const uint64_t*, uint32_t, uint32_t*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_nbhd_codes(const uint8_t*, int32_t, int32_t, int32_t, uint32_t*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_nbhd_zero(uint32_t*, uint64_t, uint32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_nbhd_scatter(const uint32_t*, int32_t, const uint32_t*, int32_t, uint32_t*,
                               uint32_t*, uint32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_nbhd_and(uint32_t*, const uint32_t*, uint64_t, uint32_t*, uint32_t, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_nbhd_sum(const uint32_t*, uint32_t, unsigned long long*, hipStream_t) {
    return hipErrorNotSupported;
}
size_t nbhd_tile_lds_bytes(uint32_t tile_words) { return tile_words * 4u; }
hipError_t launch_nbhd_tile(const uint32_t*, int32_t, const uint32_t*, const uint32_t*,
                            const uint32_t*, const uint32_t*, int32_t, uint32_t, uint32_t,
                            uint32_t*, bool, uint32_t*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_nbhd_records(const uint32_t*, int32_t, const uint32_t*, int32_t, int32_t,
                               uint32_t, uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint32_t,
                               hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_nbhd_collect(const uint32_t*, uint64_t, uint32_t*, uint64_t, unsigned long long*,
                               uint32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_nbhd_verify(const uint32_t*, uint64_t, const uint32_t*, int32_t, int32_t, int32_t,
                              int32_t, uint32_t*, uint64_t, unsigned long long*,
                              unsigned long long*, uint32_t, hipStream_t) {
    return hipErrorNotSupported;
}
const void* search_kernel_symbol() { return nullptr; }
const void* search_group_kernel_symbol(int) { return nullptr; }
hipError_t launch_search_group(const pms_dev_instance*, const pms_work_item*, uint32_t,
                               pms_dev_state*, pms_dev_counters*, const GroupQueues&, uint32_t,
                               uint32_t, hipStream_t, int, uint32_t) { return hipErrorNotSupported; }
hipError_t valu_probe(int, uint32_t, uint32_t, uint32_t*, uint64_t*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t noalloc_scratch(void** ptr, size_t* bytes) {
    *ptr = nullptr;
    *bytes = 0;
    return hipErrorNotSupported;
}
hipError_t launch_noalloc_setup(void*, const NoallocLayout&, uint32_t*, uint64_t, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_noalloc_count(const pms_dev_state*, uint64_t*, hipStream_t) {
    return hipErrorNotSupported;
}
}  // namespace pms

namespace {

int failures = 0;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

std::string random_row(std::mt19937_64& rng, int t, const char* alphabet, int k) {
    std::string r(t, 'A');
    for (auto& c : r) c = alphabet[rng() % k];
    return r;
}

// Validation of shapes and bytes.
void check_validation(std::mt19937_64& rng) {
    CHECK(validate_shape(1, 1, 1, 0) == PMS_OK);
    CHECK(validate_shape(64, 1 << 17, 16, 16) == PMS_OK);
    CHECK(validate_shape(0, 10, 4, 1) == PMS_ERR_INVALID);
    CHECK(validate_shape(65, 10, 4, 1) == PMS_ERR_INVALID);
    CHECK(validate_shape(3, 3, 4, 1) == PMS_ERR_INVALID);
    CHECK(validate_shape(3, 10, 17, 1) == PMS_ERR_INVALID);
    CHECK(validate_shape(3, 10, 4, 5) == PMS_ERR_INVALID);
    CHECK(validate_shape(3, (1 << 17) + 1, 4, 1) == PMS_ERR_INVALID);
    for (int trial = 0; trial < 200; ++trial) {
        const int n = 1 + static_cast<int>(rng() % 8), t = 1 + static_cast<int>(rng() % 300);
        std::vector<std::string> rows;
        for (int i = 0; i < n; ++i) rows.push_back(random_row(rng, t, "ACGTacgt", 8));
        const bool bad = trial % 3 == 0;
        int bi = 0, bj = 0;
        if (bad) {
            bi = static_cast<int>(rng() % n);
            bj = static_cast<int>(rng() % t);
            rows[bi][bj] = "NXU-\x01 "[rng() % 6];
        }
        std::vector<const char*> ptrs;
        for (auto& r : rows) ptrs.push_back(r.data());
        const int s = validate_rows(ptrs.data(), n, t);
        CHECK(s == (bad ? PMS_ERR_INVALID : PMS_OK));
        if (bad)
            CHECK(g_last_error.find("byte " + std::to_string(bj) + " of sequence " +
                                    std::to_string(bi)) != std::string::npos);
        // Ragged rows with N under masking.
        std::vector<int32_t> lens(n);
        std::vector<std::string> rx;
        for (int i = 0; i < n; ++i) {
            lens[i] = 1 + static_cast<int>(rng() % 200);
            rx.push_back(random_row(rng, lens[i], "ACGTN", 5));
        }
        std::vector<const char*> px;
        for (auto& r : rx) px.push_back(r.data());
        bool empty = false;
        CHECK(validate_rows_ex(px.data(), n, lens.data(), 3, PMS_INPUT_MASK_N, &empty) == PMS_OK);
        bool any_n = false;
        for (auto& r : rx) any_n |= r.find('N') != std::string::npos;
        if (any_n) CHECK(validate_rows_ex(px.data(), n, lens.data(), 3, 0, &empty) == PMS_ERR_INVALID);
    }
}

// Window strides and the output reservation.
void check_strides_and_estimates() {
    for (int l = 1; l <= 16; ++l)
        for (int t = l; t < 700; t += 7) {
            const int nw = t - l + 1;
            CHECK(window_stride(t, l, PMS_LAYOUT_PLANES) == (nw + 15) / 16 * 16);
            CHECK(window_stride(t, l, PMS_LAYOUT_BITSLICED) == (l < 2 ? 0 : (nw + 31) / 32 * 2 * l));
            for (int d = 0; d <= l; ++d) {
                const Shape s{3, t, l, d};
                const Estimate e = estimate(s);
                CHECK(std::isfinite(e.motifs) && e.motifs >= 1.0 && std::isfinite(e.visits));
                CHECK(e.visits >= 1.0 && e.visits <= 3.0 + 1e-9);
                const uint64_t cap = output_capacity(s);
                CHECK(cap >= 1 && cap <= (1ull << (2 * l)));
            }
        }
}

// Work items: every instance's range covered once, in order, on the item
// grid, within the 32-bit length field.
void check_work_plans(std::mt19937_64& rng) {
    for (int trial = 0; trial < 300; ++trial) {
        Batch b;
        const int m = 1 + static_cast<int>(rng() % 12);
        for (int i = 0; i < m; ++i) {
            const int l = 1 + static_cast<int>(rng() % 16);
            const int t = l + static_cast<int>(rng() % 900);
            const int d = static_cast<int>(rng() % (l + 1));
            b.shape.push_back(Shape{1 + static_cast<int>(rng() % 30), t, l, d});
            b.rows.push_back(nullptr);
            b.out_cap.push_back(rng() % 4 == 0 ? kCountOnly : 0);
        }
        pms_config cfg = default_config();
        cfg.chunk = 64u << (rng() % 15);
        cfg.tail_split = static_cast<uint32_t>(rng() % 65);
        cfg.variant = static_cast<uint32_t>(rng() % 4);
        plan_batch(b, cfg, 1 + rng() % 200000);
        std::vector<uint64_t> next(m, 0);
        std::vector<uint32_t> items(m, 0);
        for (const pms_work_item& w : b.work) {
            CHECK(w.inst < static_cast<uint32_t>(m));
            if (w.inst >= static_cast<uint32_t>(m)) continue;
            CHECK(w.begin == next[w.inst]);
            CHECK(w.len > 0);
            next[w.inst] = w.begin + w.len;
            items[w.inst]++;
            const uint64_t total = 1ull << (2 * b.shape[w.inst].l);
            if (total >= 4096 && w.begin + w.len < total) CHECK(w.len % 4096 == 0 && w.begin % 4096 == 0);
        }
        for (int i = 0; i < m; ++i) {
            CHECK(next[i] == (1ull << (2 * b.shape[i].l)));
            CHECK(items[i] == b.items_per_inst[i]);
        }
        size_t rows = 0;
        for (const Shape& s : b.shape) rows += s.n;
        CHECK(b.jobs.size() == rows);
        CHECK(b.off_insts < b.off_state && b.off_state < b.off_ctr && b.off_ctr < b.off_bad &&
              b.off_bad < b.off_jobs && b.off_jobs <= b.off_work && b.off_work <= b.meta_bytes);
        // The one-instance plan of the no-allocation path: closed-form items.
        const ItemPlan ip = item_plan(b.shape[0], 1.0, cfg, 1 + rng() % 200000);
        const uint64_t n_head = ip.head_end ? (ip.head_end + ip.size - 1) / ip.size : 0;
        const uint64_t h = std::min(n_head * ip.size, ip.total);
        uint64_t k = 0, count = 0, covered = 0;
        while (k < ip.total) {
            const uint64_t step = k < ip.head_end ? ip.size : ip.small;
            const uint64_t len = std::min(step, ip.total - k);
            const uint64_t begin = count < n_head ? count * ip.size : h + (count - n_head) * ip.small;
            CHECK(begin == k);
            covered += len;
            k += len;
            ++count;
        }
        CHECK(covered == ip.total);
    }
}

// Sorting of motif codes: radix path and comparison path against std::sort.
void check_sort(std::mt19937_64& rng) {
    std::vector<uint32_t> tmp;
    for (int trial = 0; trial < 60; ++trial) {
        const int bits = 2 * (1 + static_cast<int>(rng() % 16));
        const size_t k = trial < 10 ? trial : static_cast<size_t>(rng() % 30000);
        std::vector<uint32_t> v(k);
        for (auto& x : v) x = static_cast<uint32_t>(rng()) & (bits == 32 ? ~0u : ((1u << bits) - 1));
        std::vector<uint32_t> want = v;
        std::sort(want.begin(), want.end());
        sort_codes(v.data(), v.size(), bits, tmp);
        CHECK(v == want);
    }
}

// The autotune cache file and its key.
void check_cache(const char* dir) {
    const std::string path = std::string(dir) + "/tune.json";
    std::remove(path.c_str());
    pms_config a{8192, 2, 0, 8, 3, 1}, b{16384, 4, 0, 0, 0, 2}, got{};
    CHECK(!cache_lookup(path, "k1", &got));
    cache_store(path, "k1", a);
    cache_store(path, "k2", b);
    cache_store(path, "k1", b);
    CHECK(cache_lookup(path, "k1", &got) && got.chunk == b.chunk && got.filter == b.filter);
    CHECK(cache_lookup(path, "k2", &got) && got.wg_waves == b.wg_waves);
    CHECK(!cache_lookup(path, "k3", &got));
    Ctx c;
    c.arch = "gfx950";
    c.cus = 256;
    const std::string key = tune_key(c, 20, 600, 15, 4);
    CHECK(key.find("gfx950/cu256/") != std::string::npos && key.find("/l15/d4/n20/") != std::string::npos);
}

// The C ABI's host-side error paths; with no device, valid calls report a
// device error and write nothing.
void check_fill_work_items() {
    pms_work_item w[8];
    CHECK(pms_fill_work_items(4096, 64 * 5 + 7, 64, 3, w, 8) == 6);
    CHECK(w[0].begin == 4096 && w[0].len == 64 && w[0].inst == 3);
    CHECK(w[5].begin == 4096 + 64 * 5 && w[5].len == 7);
    CHECK(pms_fill_work_items(0, 1000, 64, 1, w, 8) == 8 && w[7].begin == 448);
    CHECK(pms_fill_work_items(0, 0, 64, 1, w, 8) == 0);
    CHECK(pms_fill_work_items(0, 10, 0, 1, w, 8) == -1);
    CHECK(pms_fill_work_items(0, 10, 64, 1, nullptr, 8) == -1);
    CHECK(pms_fill_work_items(1, 1ull << 32, 64, 1, w, 8) == -1);
    CHECK(pms_fill_work_items(0, 1ull << 32, 1u << 31, 1, w, 8) == 2 && w[1].len == (1u << 31));
}

void check_abi() {
    uint32_t out[4] = {7, 7, 7, 7};
    uint64_t cnt = 4;
    const char* rows[2] = {"ACGTACGT", "ACGTNCGT"};
    CHECK(pms_solve(nullptr, 1, 8, 4, 1, out, &cnt) == PMS_ERR_INVALID && cnt == 0);
    cnt = 4;
    CHECK(pms_solve(rows, 2, 8, 4, 1, out, &cnt) == PMS_ERR_INVALID && cnt == 0);
    CHECK(out[0] == 7);
    cnt = 4;
    const int s = pms_solve(rows, 1, 8, 4, 1, out, &cnt);
    CHECK(s == PMS_ERR_DEVICE || s == PMS_OK);
    CHECK(std::string(pms_status_string(PMS_ERR_OVERFLOW)) == "output capacity exceeded");
    char buf[8];
    pms_decode(0b11100100u, 4, buf);
    CHECK(std::string(buf, 4) == "TGCA");
    pms_config cfg{100, 0, 0, 0, 0, 0};
    CHECK(pms_set_config(&cfg) == PMS_ERR_INVALID);
    CHECK(pms_set_config(nullptr) == PMS_OK);
    pms_result res[2];
    pms_instance inst[2] = {{rows, 2, 8, 4, 1, out, 4}, {rows, 1, 8, 9, 1, out, 4}};
    CHECK(pms_solve_many(inst, 2, res) == PMS_ERR_INVALID);
    CHECK(res[0].status == PMS_ERR_INVALID && res[1].status == PMS_ERR_INVALID);
    CHECK(pms_shutdown() == PMS_OK);
}

}  // namespace

int main(int argc, char** argv) {
    std::mt19937_64 rng(1403);
    check_validation(rng);
    check_strides_and_estimates();
    check_work_plans(rng);
    check_sort(rng);
    check_cache(argc > 1 ? argv[1] : "/tmp");
    check_abi();
    check_fill_work_items();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
