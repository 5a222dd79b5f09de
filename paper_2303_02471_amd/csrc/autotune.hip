// Autotuner: picks spgemm_options for a workload by timing a few candidate
// settings of the accumulator thresholds (the role of the paper's switch
// threshold t, Section 3.3, and its size adaptation, Section 3.2), and keeps
// the choice in a JSON cache keyed by device and workload signature.
//
// Options only decide which accumulator takes a column; every accumulator
// computes Algorithm 1's values bit for bit, so tuning never changes results.
//
// Search: coordinate descent from the defaults over t_esc, t_block, t_split,
// hash_cap and dense_rows; a candidate replaces the current best when it is at least 2%
// faster. Each candidate is timed as symbolic + numeric, best of three runs
// after one warm-up run.
//
// Cache file: {"spgemm_tune_cache": 1, "entries": [{"key": "...", "t_esc": ..,
// "t_dense": .., "dense_rows": .., "hash_cap": .., "t_split": .., "t_block": ..,
// "ms": ..}, ...]}. A file that does not parse as such is treated as empty and
// is rewritten by the next store.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/spgemm.h"

namespace {

// ---------------------------------------------------------------- cache JSON
struct Entry {
    std::string key;
    spgemm_options o{};
    double ms = 0.0;
};

// Minimal reader for the cache schema (objects, arrays, strings without
// escapes other than \" and \\, numbers, true/false/null).
struct Reader {
    const char *p, *end;
    bool ok = true;
    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool eat(char c) {
        ws();
        if (p < end && *p == c) { ++p; return true; }
        return false;
    }
    bool str(std::string &out) {
        ws();
        if (p >= end || *p != '"') return ok = false;
        ++p;
        out.clear();
        while (p < end && *p != '"') {
            if (*p == '\\') {
                if (++p >= end) return ok = false;
                if (*p != '"' && *p != '\\') return ok = false;
            }
            out.push_back(*p++);
        }
        if (p >= end) return ok = false;
        ++p;
        return true;
    }
    bool num(double &out) {
        ws();
        char *e = nullptr;
        out = std::strtod(p, &e);
        if (e == p || e > end) return ok = false;
        p = e;
        return true;
    }
    bool skip_value() {
        ws();
        if (p >= end) return ok = false;
        if (*p == '"') { std::string s; return str(s); }
        if (*p == '{' || *p == '[') {
            const char close = *p == '{' ? '}' : ']';
            const bool obj = *p == '{';
            ++p;
            if (eat(close)) return true;
            do {
                if (obj) {
                    std::string k;
                    if (!str(k) || !eat(':')) return ok = false;
                }
                if (!skip_value()) return false;
            } while (eat(','));
            return eat(close) || (ok = false);
        }
        for (const char *w : {"true", "false", "null"}) {
            const size_t n = std::strlen(w);
            if ((size_t)(end - p) >= n && std::strncmp(p, w, n) == 0) { p += n; return true; }
        }
        double d;
        return num(d);
    }
    bool entry(Entry &e) {
        if (!eat('{')) return ok = false;
        bool have_key = false;
        if (eat('}')) return ok = false;
        do {
            std::string k;
            if (!str(k) || !eat(':')) return ok = false;
            if (k == "key") {
                if (!str(e.key)) return false;
                have_key = true;
                continue;
            }
            double v;
            int32_t *f = nullptr;
            if (k == "t_esc") f = &e.o.t_esc;
            else if (k == "t_dense") f = &e.o.t_dense;
            else if (k == "dense_rows") f = &e.o.dense_rows;
            else if (k == "hash_cap") f = &e.o.hash_cap;
            else if (k == "t_split") f = &e.o.t_split;
            else if (k == "t_block") f = &e.o.t_block;
            if (f || k == "ms") {
                if (!num(v)) return false;
                if (f) {
                    if (v != std::floor(v) || std::fabs(v) > 1e9) return ok = false;
                    *f = (int32_t)v;
                } else {
                    e.ms = v;
                }
            } else if (!skip_value()) {
                return false;
            }
        } while (eat(','));
        if (!eat('}')) return ok = false;
        return have_key || (ok = false);
    }
    // whole file
    bool file(std::vector<Entry> &out) {
        if (!eat('{')) return ok = false;
        bool marked = false, have_entries = false;
        if (eat('}')) return ok = false;
        do {
            std::string k;
            if (!str(k) || !eat(':')) return ok = false;
            if (k == "spgemm_tune_cache") {
                double v;
                if (!num(v) || v != 1.0) return ok = false;
                marked = true;
            } else if (k == "entries") {
                if (!eat('[')) return ok = false;
                have_entries = true;
                if (!eat(']')) {
                    do {
                        Entry e;
                        if (!entry(e)) return false;
                        out.push_back(e);
                    } while (eat(','));
                    if (!eat(']')) return ok = false;
                }
            } else if (!skip_value()) {
                return false;
            }
        } while (eat(','));
        if (!eat('}')) return ok = false;
        ws();
        return (marked && have_entries && p == end) || (ok = false);
    }
};

bool load_cache(const char *path, std::vector<Entry> &out) {
    out.clear();
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, n);
        if (text.size() > (64u << 20)) break;  // not a cache of this library
    }
    std::fclose(f);
    Reader r{text.data(), text.data() + text.size()};
    if (!r.file(out) || !r.ok) {
        out.clear();
        return false;
    }
    return true;
}

std::string quote(const std::string &s) {
    std::string q = "\"";
    for (char c : s) {
        if (c == '"' || c == '\\') q.push_back('\\');
        q.push_back(c);
    }
    return q + "\"";
}

bool save_cache(const char *path, const std::vector<Entry> &es) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\"spgemm_tune_cache\": 1, \"entries\": [");
    for (size_t i = 0; i < es.size(); ++i) {
        const Entry &e = es[i];
        std::fprintf(f,
                     "%s\n  {\"key\": %s, \"t_esc\": %d, \"t_dense\": %d, \"dense_rows\": %d, "
                     "\"hash_cap\": %d, \"t_split\": %d, \"t_block\": %d, \"ms\": %.6g}",
                     i ? "," : "", quote(e.key).c_str(), e.o.t_esc, e.o.t_dense, e.o.dense_rows,
                     e.o.hash_cap, e.o.t_split, e.o.t_block, e.ms);
    }
    std::fprintf(f, "\n]}\n");
    const bool good = std::fflush(f) == 0;
    std::fclose(f);
    if (!good || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

// half-octave bucket of a size: similar workloads share a cache entry
int bucket(long long x) { return x <= 0 ? -1 : (int)std::floor(2.0 * std::log2((double)x)); }

// ---------------------------------------------------------------- trials
struct Trial {
    int count;
    const spgemm_csc *A, *B;
    spgemm_dtype dt;
    hipStream_t s;
    std::vector<int32_t *> cp, ri;
    std::vector<void *> cv;
    std::vector<int64_t> nnz;
    void *cbuf = nullptr;

    ~Trial() {
        if (cbuf) (void)hipFree(cbuf);
    }

    spgemm_status run_once(const spgemm_options &o, spgemm_plan *plan) {
        spgemm_status st;
        if (count == 1) {
            st = spgemm_symbolic(A, B, dt, &o, s, plan, cp[0], nnz.data());
            if (st) return st;
            return spgemm_numeric(*plan, A[0].val, B[0].val, ri[0], cv[0], s);
        }
        st = spgemm_batched(count, A, B, dt, &o, s, plan, cp.data(), nnz.data(), nullptr, nullptr);
        if (st) return st;
        return spgemm_batched(count, A, B, dt, &o, s, plan, cp.data(), nnz.data(), ri.data(),
                              cv.data());
    }

    // output arrays sized by a first symbolic run (nnz(C) does not depend
    // on the options): column pointers and C of every problem in one buffer
    spgemm_status setup(const spgemm_options &o) {
        auto carve_cp = [&](char *q) {
            cp.resize(count);
            for (int i = 0; i < count; ++i) {
                cp[i] = (int32_t *)q;
                q += (4 * ((size_t)B[i].ncols + 1) + 255) / 256 * 256;
            }
            return q;
        };
        size_t cpb = 0;
        for (int i = 0; i < count; ++i) cpb += (4 * ((size_t)B[i].ncols + 1) + 255) / 256 * 256;
        if (hipMalloc(&cbuf, cpb) != hipSuccess) return SPGEMM_ERR_NO_MEMORY;
        carve_cp((char *)cbuf);
        nnz.assign(count, 0);
        spgemm_plan plan = nullptr;
        const spgemm_status st =
            count == 1 ? spgemm_symbolic(A, B, dt, &o, s, &plan, cp[0], nnz.data())
                       : spgemm_batched(count, A, B, dt, &o, s, &plan, cp.data(), nnz.data(),
                                        nullptr, nullptr);
        spgemm_plan_destroy(plan);
        (void)hipFree(cbuf);
        cbuf = nullptr;
        if (st) return st;
        const size_t vb = dt == SPGEMM_F64 ? 8 : 4;
        size_t out = 0;
        for (int i = 0; i < count; ++i)
            out += (4 * (size_t)nnz[i] + 255) / 256 * 256 + (vb * (size_t)nnz[i] + 255) / 256 * 256;
        if (hipMalloc(&cbuf, cpb + out) != hipSuccess) return SPGEMM_ERR_NO_MEMORY;
        char *q = carve_cp((char *)cbuf);
        ri.resize(count);
        cv.resize(count);
        for (int i = 0; i < count; ++i) {
            ri[i] = (int32_t *)q;
            q += (4 * (size_t)nnz[i] + 255) / 256 * 256;
            cv[i] = q;
            q += (vb * (size_t)nnz[i] + 255) / 256 * 256;
        }
        return SPGEMM_OK;
    }

    // best of three timed runs after one warm-up, in ms
    spgemm_status time(const spgemm_options &o, double &ms) {
        spgemm_plan plan = nullptr;
        spgemm_status st = run_once(o, &plan);
        if (!st && hipStreamSynchronize(s) != hipSuccess) st = SPGEMM_ERR_HIP;
        ms = 1e30;
        for (int r = 0; r < 3 && !st; ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            st = run_once(o, &plan);
            if (!st && hipStreamSynchronize(s) != hipSuccess) st = SPGEMM_ERR_HIP;
            const auto t1 = std::chrono::steady_clock::now();
            ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        spgemm_plan_destroy(plan);
        return st;
    }
};

spgemm_options defaults() {
    spgemm_options o{};
    o.t_esc = 256;
    o.t_dense = 1;
    o.dense_rows = 0;
    o.hash_cap = 0;
    o.t_split = 2048;
    o.t_block = 0;
    return o;
}

// option values a cache entry may hold (the ranges spgemm_symbolic accepts)
bool usable(const spgemm_options &o) {
    return o.t_esc >= 4 && o.t_esc <= 256 && o.t_dense >= 1 && o.dense_rows >= 0 &&
           (o.hash_cap == 0 || (o.hash_cap >= 16 && o.hash_cap <= (1 << 20))) &&
           (o.t_split == -1 || o.t_split >= 1) && o.t_block >= -1;
}

}  // namespace

extern "C" {

spgemm_status spgemm_tune_key(int32_t count, const spgemm_csc *A_host, const spgemm_csc *B_host,
                              spgemm_dtype dt, const char *device_tag, char *key_out,
                              int32_t key_len) {
    if (!A_host || !B_host || !device_tag || !key_out) return SPGEMM_ERR_NULL;
    if (count < 1 || key_len < 1) return SPGEMM_ERR_INVALID;
    if (dt != SPGEMM_F32 && dt != SPGEMM_F64) return SPGEMM_ERR_DTYPE;
    long long m = 0, k = 0, n = 0, za = 0, zb = 0;
    for (int i = 0; i < count; ++i) {
        m += A_host[i].nrows;
        k += A_host[i].ncols;
        n += B_host[i].ncols;
        za += A_host[i].nnz;
        zb += B_host[i].nnz;
    }
    char buf[512];
    const int w = std::snprintf(buf, sizeof buf, "%s|%s|p%d|m%d|k%d|n%d|a%d|b%d", device_tag,
                                dt == SPGEMM_F64 ? "f64" : "f32", bucket(count), bucket(m),
                                bucket(k), bucket(n), bucket(za), bucket(zb));
    if (w < 0 || w >= key_len) return SPGEMM_ERR_INVALID;
    std::memcpy(key_out, buf, (size_t)w + 1);
    return SPGEMM_OK;
}

spgemm_status spgemm_tune_cache_load(const char *path, const char *key, spgemm_options *opts_out) {
    if (!path || !key || !opts_out) return SPGEMM_ERR_NULL;
    std::vector<Entry> es;
    if (!load_cache(path, es)) return SPGEMM_ERR_NOT_TUNED;
    for (const Entry &e : es) {
        if (e.key != key) continue;
        // values outside the options' ranges make the entry unusable
        if (!usable(e.o)) return SPGEMM_ERR_NOT_TUNED;
        *opts_out = defaults();
        opts_out->t_esc = e.o.t_esc;
        opts_out->t_dense = e.o.t_dense;
        opts_out->dense_rows = e.o.dense_rows;
        opts_out->hash_cap = e.o.hash_cap;
        opts_out->t_split = e.o.t_split;
        opts_out->t_block = e.o.t_block;
        return SPGEMM_OK;
    }
    return SPGEMM_ERR_NOT_TUNED;
}

spgemm_status spgemm_tune_cache_store(const char *path, const char *key,
                                      const spgemm_options *opts, double ms) {
    if (!path || !key || !opts) return SPGEMM_ERR_NULL;
    std::vector<Entry> es;
    (void)load_cache(path, es);  // an unreadable or corrupt file is replaced
    Entry ne;
    ne.key = key;
    ne.o = *opts;
    ne.o.flags = 0;
    ne.ms = ms;
    bool found = false;
    for (Entry &e : es)
        if (e.key == ne.key) {
            e = ne;
            found = true;
        }
    if (!found) es.push_back(ne);
    return save_cache(path, es) ? SPGEMM_OK : SPGEMM_ERR_INVALID;
}

spgemm_status spgemm_autotune(int32_t count, const spgemm_csc *A_host, const spgemm_csc *B_host,
                              spgemm_dtype dt, void *stream, const char *cache_path,
                              uint32_t tune_flags, spgemm_options *opts_out,
                              spgemm_tune_report *report_out) {
    if (!A_host || !B_host || !opts_out) return SPGEMM_ERR_NULL;
    if (count < 1) return SPGEMM_ERR_INVALID;
    if (dt != SPGEMM_F32 && dt != SPGEMM_F64) return SPGEMM_ERR_DTYPE;
    spgemm_tune_report rep{};
    // device tag: architecture and compute units
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return SPGEMM_ERR_HIP;
    char tag[160];
    std::snprintf(tag, sizeof tag, "%s:%d", prop.gcnArchName, prop.multiProcessorCount);
    char key[512];
    spgemm_status st = spgemm_tune_key(count, A_host, B_host, dt, tag, key, sizeof key);
    if (st) return st;
    if (cache_path && !(tune_flags & SPGEMM_TUNE_REFRESH)) {
        if (spgemm_tune_cache_load(cache_path, key, opts_out) == SPGEMM_OK) {
            rep.from_cache = 1;
            if (report_out) *report_out = rep;
            return SPGEMM_OK;
        }
    }
    if (tune_flags & SPGEMM_TUNE_LOOKUP_ONLY) return SPGEMM_ERR_NOT_TUNED;
    for (int i = 0; i < count; ++i)
        if ((A_host[i].nnz > 0 && !A_host[i].val) || (B_host[i].nnz > 0 && !B_host[i].val))
            return SPGEMM_ERR_NULL;

    Trial tr{count, A_host, B_host, dt, (hipStream_t)stream};
    spgemm_options best = defaults();
    if ((st = tr.setup(best))) return st;
    double best_ms;
    if ((st = tr.time(best, best_ms))) return st;
    rep.default_ms = best_ms;
    rep.trials = 1;
    long long m_max = 0;
    for (int i = 0; i < count; ++i) m_max = std::max<long long>(m_max, A_host[i].nrows);
    struct Axis {
        int32_t spgemm_options::*field;
        std::vector<int32_t> values;
    };
    std::vector<Axis> axes = {
        {&spgemm_options::t_esc, {128, 64, 32}},
        {&spgemm_options::t_block, {4096}},
        {&spgemm_options::t_split, {1024, 4096, -1}},
        {&spgemm_options::hash_cap, {2048, 1024}},
    };
    // direct indexing applies only when a window's rows fit the LDS table
    if (m_max <= 16384) axes.push_back({&spgemm_options::dense_rows, {1}});
    for (const Axis &ax : axes) {
        spgemm_options cur = best;
        for (int32_t v : ax.values) {
            spgemm_options cand = cur;
            cand.*ax.field = v;
            double ms;
            if ((st = tr.time(cand, ms))) return st;
            ++rep.trials;
            if (ms < 0.98 * best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
    }
    rep.best_ms = best_ms;
    *opts_out = best;
    if (cache_path) (void)spgemm_tune_cache_store(cache_path, key, &best, best_ms);
    if (report_out) *report_out = rep;
    return SPGEMM_OK;
}

}  // extern "C"
