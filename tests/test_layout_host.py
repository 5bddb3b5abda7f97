"""Host checks of the block layout (the header shared by the host launcher
and the block kernel), compiled with the host C++ compiler: no GPU needed.

The layout decides what fits in a CU's LDS and where the level sort's
histogram lies; the kernel relies on these properties.
"""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_04669_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <initializer_list>
#include "pss_layout.h"
using namespace pss;
int main() {
    printf("[");
    bool first = true;
    auto emit = [&](unsigned k, unsigned g) {
        for (unsigned sx : {0u, 32u, 48u, 64u}) {
            ChunkLayout L = ChunkLayout::make(k, g != 0, sx);
            printf("%s{\"k\":%u,\"g\":%u,\"sx\":%u,\"nb\":%u,\"ts\":%u,\"slots\":%u,\"table\":%u,\"list\":%u,"
                   "\"tkey\":%u,\"list2\":%u,\"tkey2\":%u,\"state\":%u,\"ring\":%u,\"hist\":%u,\"lds\":%u,"
                   "\"es\":%u,\"lanes\":%u,\"ch\":%u}",
                   first ? "" : ",", k, g, sx, L.nbuckets, L.tsize, L.slots, L.off_table, L.off_list, L.off_tkey,
                   L.off_list2, L.off_tkey2, L.state_bytes, L.off_ring, L.off_hist, L.lds_bytes, L.err_stride,
                   sort_lanes_per_k(k), L.choices);
            first = false;
        }
    };
    for (unsigned g = 0; g < 2; ++g) {
        for (unsigned k = 2; k <= 70000; k = k < 600 ? k + 1 : k + 37)
            if (g || k <= 8192) emit(k, g);
        for (unsigned k : {1000u, 1024u, 1025u, 2000u, 2048u, 4096u, 10000u, 50000u})
            if (g || k <= 8192) emit(k, g);
    }
    printf("]\n");
    // error widths at the boundaries: blocks of 255 k - 1, 255 k, 65535 k - 1, 65535 k items
    for (unsigned k : {2u, 500u, 2000u, 50000u}) {
        ChunkLayout L = ChunkLayout::make(k, k > 4096);
        printf("%u %u %u %u %u ", L.err_bytes, L.with_error_width(255ull * k - 1).err_bytes,
               L.with_error_width(255ull * k).err_bytes, L.with_error_width(65535ull * k - 1).err_bytes,
               L.with_error_width(65535ull * k).err_bytes);
    }
    printf("\n");
    // packed errors: err_bytes and count mask either side of the bounds, LDS and device-memory state
    for (unsigned k : {64u, 4096u, 10000u}) {
        const ChunkLayout L = ChunkLayout::make(k, k > 4096);
        for (unsigned long long mb : {1023ull * k - 1, 1023ull * k, (unsigned long long)kCountMask,
                                      (unsigned long long)kCountMask + 1}) {
            const ChunkLayout P = L.with_error_width(mb, true), Q = L.with_error_width(mb);
            printf("%u %llu %u %u %u %u ", k, mb, P.err_bytes, P.count_mask, Q.err_bytes, Q.count_mask);
        }
    }
    printf("\n");
    printf("%u %u %u %llu %u %u\n", kBucketSlots, kStash, kHistBytes, (unsigned long long)kStreamBound, kRing, kLdsUnit);
    for (unsigned b : {1u, 1280u, 1281u, 11520u, 11600u, 32000u, 32608u})
        printf("%u ", lds_waves(163840, b));
    printf("\n");
    // the Frequent block layout beside the Space Saving one of the same k
    auto emit_freq = [](unsigned k) {
        const FreqLayout F = FreqLayout::make(k);
        const ChunkLayout L = ChunkLayout::make(k, false);
        printf("%u %u %u %u %u %u %u %u %u ", k, F.choices, L.choices, F.nbuckets, L.nbuckets, F.slots,
               F.off_ring, F.lds_bytes, lds_waves(163840, F.lds_bytes));
    };
    for (unsigned k = 2; k <= 8192; k += k < 600 ? 1 : 37) emit_freq(k);
    for (unsigned k : {1000u, 1024u, 1025u, 2000u, 2048u, 4096u}) emit_freq(k);
    printf("\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def layouts(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("layout")
    src = d / "layout.cpp"
    src.write_text(PROGRAM)
    exe = d / "layout"
    cc = subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], capture_output=True,
                        text=True)
    assert cc.returncode == 0, cc.stderr
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines()
    c = {"ewidth": [int(v) for v in out[1].split()]}
    pk = [int(v) for v in out[2].split()]
    c["packing"] = [dict(zip(["k", "mb", "pbytes", "pmask", "bytes", "mask"], pk[i:i + 6]))
                    for i in range(0, len(pk), 6)]
    consts = [int(v) for v in out[3].split()]
    c.update(zip(["bucket", "stash", "hist", "bound", "ring", "unit"], consts))
    c["waves"] = [int(v) for v in out[4].split()]
    f = [int(v) for v in out[5].split()]
    c["freq"] = [dict(zip(["k", "ch", "ch_ss", "nb", "nb_ss", "slots", "ring", "lds", "waves"], f[i:i + 9]))
                 for i in range(0, len(f), 9)]
    return json.loads(out[0]), c


def test_regions_are_disjoint_and_sized(layouts):
    rows, c = layouts
    for r in rows:
        k, slots = r["k"], r["slots"]
        idx = 4 if r["g"] else 2
        assert r["ts"] == c["bucket"] * r["nb"] and slots == r["ts"] + c["stash"]
        assert slots >= k + 64  # every counter plus a full window of claims has a slot
        assert r["nb"] >= 2  # two distinct buckets per item
        assert r["table"] == 0
        assert r["list"] >= 8 * slots
        assert r["tkey"] >= r["list"] + idx * k
        if r["g"]:
            # the radix sort's ids and ping-pong buffers
            assert r["list2"] >= r["tkey"] + 4 * k and r["tkey2"] >= r["list2"] + 4 * k
            assert r["state"] >= r["tkey2"] + 4 * k
            assert r["ring"] == 0  # LDS holds only the ring and the histogram
        else:
            # the LDS sorts read ids from the table: no id buffer
            assert r["state"] == r["tkey"] == r["list2"] == r["tkey2"]
            assert r["ring"] >= r["state"]
        assert r["lds"] >= r["ring"] + 4 * c["ring"]
        for off in ("list", "tkey", "state", "ring", "hist", "lds"):
            assert r[off] % 16 == 0, (off, r)
        assert r["es"] % 32 == 0 and r["es"] >= slots


def test_histogram_over_the_list_with_state_in_lds(layouts):
    # the LDS sorts hold the list in registers while the histogram is in use
    rows, c = layouts
    for r in rows:
        if not r["g"]:
            assert r["hist"] == r["list"]
            assert r["tkey"] - r["list"] >= c["hist"]  # the list region holds the histogram
        else:
            assert r["hist"] >= r["ring"] + 4 * c["ring"] and r["lds"] >= r["hist"] + c["hist"]


def test_footprint_grows_with_k_inside_a_class(layouts):
    # a batched launch sizes every wave's LDS slab by the largest k of its class
    rows, _ = layouts
    by = {}
    for r in rows:
        if not r["g"]:
            by.setdefault((r["sx"], r["lanes"]), []).append((r["k"], r["lds"]))
    for v in by.values():
        v.sort()
        assert all(a[1] <= b[1] for a, b in zip(v, v[1:]))


def test_lds_units(layouts):
    # 1280-byte units out of 160 KiB, as measured on MI355X with one-wave workgroups
    _, c = layouts
    assert c["unit"] == 1280
    assert c["waves"] == [128, 128, 64, 14, 12, 5, 4]


def test_benchmark_sizes_fit_their_wave_counts(layouts):
    rows, c = layouts
    lds = {(r["k"], r["sx"]): r["lds"] for r in rows if not r["g"]}

    def waves(b):
        return (160 * 1024) // (-(-b // c["unit"]) * c["unit"])

    assert waves(lds[(500, 0)]) >= 16
    assert waves(lds[(2000, 0)]) >= 6


def test_stream_bound_leaves_room_for_the_window_tags(layouts):
    _, c = layouts
    # two tag ranges of 64 values (victim ranks, claiming lanes) above every count
    assert c["bound"] == (1 << 32) - 128


def test_error_width_holds_every_error(layouts):
    # an error is at most (block length) / k: bytes below 255 k items per
    # block, 16 bits below 65535 k, else 32 bits; make() keeps 32 bits
    _, c = layouts
    assert c["ewidth"] == [4, 1, 2, 2, 4] * 4


def test_three_bucket_choices_only_for_the_large_lds_classes(layouts):
    # the block kernels derive the same number from their register class
    rows, c = layouts
    for r in rows:
        want = 3 if (not r["g"] and r["lanes"] >= 32) else 2
        assert r["ch"] == want, r
        # every item has that many distinct buckets beyond the ones id 0 takes
        assert r["nb"] > r["ch"]


def test_frequent_layout_shares_the_table_shape(layouts):
    # the Frequent block kernel uses the Space Saving table of the same k:
    # the same buckets per item and bucket count, the 64-slot stash after
    # them, the 8-byte entries before the ring
    _, c = layouts
    for r in c["freq"]:
        assert r["ch"] == r["ch_ss"] and r["nb"] == r["nb_ss"], r
        assert r["slots"] == 8 * r["nb"] + c["stash"] and r["ring"] >= 8 * r["slots"], r
        assert r["lds"] == r["ring"] + 4 * c["ring"], r
    # three choices above k = 1024 keep 7 blocks per CU up to k = 2048
    # (two would leave 5 at k = 2000)
    for r in c["freq"]:
        if 1024 < r["k"] <= 2048:
            assert r["ch"] == 3 and r["waves"] >= 7, r
    assert {r["k"]: r["waves"] for r in c["freq"]}[2000] == 7


def test_errors_pack_into_count_words_only_within_bounds(layouts):
    # packed (err_bytes 0, counts in the low 22 bits) when the state is in
    # LDS, blocks hold at most 2^22 - 1 items and floor(block / k) <= 1022;
    # never unless the caller allows it, never with the state in device memory
    _, c = layouts
    full, low22 = 0xFFFFFFFF, (1 << 22) - 1
    for r in c["packing"]:
        want = r["k"] <= 4096 and r["mb"] <= low22 and r["mb"] // r["k"] <= 1022
        assert (r["pbytes"], r["pmask"]) == ((0, low22) if want else (r["bytes"], full)), r
        assert r["bytes"] in (1, 2, 4) and r["mask"] == full, r
    by = {(r["k"], r["mb"]): r["pbytes"] for r in c["packing"]}
    assert by[(64, 1023 * 64 - 1)] == 0 and by[(64, 1023 * 64)] == 2
    assert by[(4096, 1023 * 4096 - 1)] == 0 and by[(4096, 1023 * 4096)] == 2
    assert all(by[(10000, mb)] != 0 for (k, mb) in by if k == 10000)


def test_level_histogram_fits_the_list_area(layouts):
    # the bucketed level sort lays its histogram over the list: 257 words,
    # 513 for levels of over 1024 counters (9-bit digits), which only blocks
    # with k > 1024 (32 sort lanes per k) list
    rows, _ = layouts
    for r in rows:
        if r["g"]:
            continue
        area = r["tkey"] - r["list"]
        assert area >= 4 * 257, r
        if r["lanes"] >= 32:
            assert area >= 4 * 513, r
