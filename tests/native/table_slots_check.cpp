// Host-only check of the library's table-capacity helpers at the sizes where
// 32-bit slot arithmetic ends.  Prints one "name value" line per case; a
// refused size prints "name unsupported".  Built and run by test_capacity.py.
#include <cstdio>

#include "bsim_internal.h"

static void show(const char* name, uint64_t want, uint64_t min_slots) {
    try {
        std::printf("%s %llu\n", name, static_cast<unsigned long long>(bsim::table_slots(want, min_slots, name)));
    } catch (const bsim::DeviceError& e) {
        std::printf("%s unsupported %d\n", name, e.status);
    }
}

static void show_split(const char* name, uint64_t n) {
    try {
        std::printf("%s %llu\n", name, static_cast<unsigned long long>(bsim::split_table_slots(n)));
    } catch (const bsim::DeviceError& e) {
        std::printf("%s unsupported %d\n", name, e.status);
    }
}

int main() {
    std::printf("next_pow2_2e32p1 %llu\n", static_cast<unsigned long long>(bsim::next_pow2((1ull << 32) + 1)));
    // change detection: next_pow2(2 m + 2) slots per snapshot
    show("diff_m_2e30", 2ull * (1ull << 30) + 2, 64);            // 2^31 + 2 -> 2^32 slots
    show("diff_m_2e31m2", 2ull * ((1ull << 31) - 2) + 2, 64);    // 2^32 - 2 -> 2^32 slots
    show("diff_m_2e31m1", 2ull * ((1ull << 31) - 1) + 2, 64);    // 2^32 -> 2^32 slots
    show("diff_m_2e31", 2ull * (1ull << 31) + 2, 64);            // needs 2^33: refused
    show("diff_m_0", 2, 64);
    // class tables: next_pow2(1.5 n + 1), at least 64 slots
    show_split("split_n_0", 0);
    show_split("split_n_2e27", 1ull << 27);                      // 2^28 slots
    show_split("split_n_1431655765", 1431655765ull);             // n + n/2 + 1 = 2^31: 2^31 slots
    show_split("split_n_1431655766", 1431655766ull);             // just past 2^31: 2^32 slots
    show_split("split_n_2863311530", 2863311530ull);             // 1.5 n + 1 = 2^32: 2^32 slots
    show_split("split_n_2863311531", 2863311531ull);             // just past: refused
    show_split("split_n_4294967294", 4294967294ull);             // largest n: refused
    return 0;
}
