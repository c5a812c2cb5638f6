// Persisted autotune table (bfs_tune_table_*): JSON lines, one flat object
// per (graph, device, mode) with integer fields and the tuned time.  Only
// files of this form are read; any line that does not parse is skipped.
#include <fcntl.h>
#include <sys/file.h>
#include <unistd.h>

#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <string>
#include <vector>

#include "hybfs_internal.h"

namespace hybfs {
namespace {

std::mutex g_table_mu;   // puts in one process, one at a time

// Exclusive advisory lock on "<path>.lock" for the lifetime of the object, so
// that puts from different processes do not overwrite each other's entries
// (each reads the table, then renames its rewritten copy over it).
struct FileLock {
    int fd = -1;
    int err = 0;   // errno of a failed open or lock
    explicit FileLock(const std::string &path)
    {
        fd = open((path + ".lock").c_str(), O_RDWR | O_CREAT | O_CLOEXEC, 0644);
        if (fd < 0) {
            err = errno;
            return;
        }
        int rc;
        do rc = flock(fd, LOCK_EX);
        while (rc != 0 && errno == EINTR);
        if (rc != 0) {
            err = errno;
            close(fd);
            fd = -1;
        }
    }
    ~FileLock()
    {
        if (fd >= 0) {
            flock(fd, LOCK_UN);
            close(fd);
        }
    }
};

// The tuned fields, in file order.
struct Field {
    const char *name;
    int32_t bfs_options::*member;
};
const Field kTuned[] = {
    {"alpha", &bfs_options::alpha},
    {"beta", &bfs_options::beta},
    {"probe_k", &bfs_options::probe_k},
    {"td_hub_degree", &bfs_options::td_hub_degree},
    {"grid_blocks", &bfs_options::grid_blocks},
    {"words_per_wave", &bfs_options::words_per_wave},
    {"bu_serial_probes", &bfs_options::bu_serial_probes},
    {"alpha_binned", &bfs_options::alpha_binned},
};

// The number after "name": on the line; false when absent or malformed.
bool field(const std::string &line, const char *name, double *out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    const char *s = line.c_str() + p + pat.size();
    char *end = nullptr;
    errno = 0;
    const double v = std::strtod(s, &end);
    if (end == s || errno != 0 || !std::isfinite(v)) return false;
    *out = v;
    return true;
}

bool field_i64(const std::string &line, const char *name, int64_t *out)
{
    double v;
    if (!field(line, name, &v) || v != std::floor(v) || std::fabs(v) > 9.0e15) return false;
    *out = (int64_t)v;
    return true;
}

bool same_key(const std::string &line, const bfs_tune_key &k)
{
    int64_t n, nnz, md, iso, cus, mode;
    return field_i64(line, "n", &n) && field_i64(line, "nnz", &nnz) && field_i64(line, "max_degree", &md) &&
           field_i64(line, "isolated", &iso) && field_i64(line, "cus", &cus) && field_i64(line, "mode", &mode) &&
           n == k.n && nnz == k.nnz && md == k.max_degree && iso == k.isolated && cus == k.cus && mode == k.mode;
}

// The options of a line on top of `base`; false when a field is missing or
// the result is not a valid option set.
bool line_options(const std::string &line, const bfs_options &base, bfs_options *out, double *best_us)
{
    bfs_options o = base;
    for (const Field &f : kTuned) {
        int64_t v;
        if (!field_i64(line, f.name, &v) || v < INT32_MIN || v > INT32_MAX) return false;
        o.*(f.member) = (int32_t)v;
    }
    double t = 0.0;
    if (!field(line, "best_us", &t)) return false;
    if (validate_options(o) != BFS_OK) {
        clear_error();
        return false;
    }
    *out = o;
    *best_us = t;
    return true;
}

std::string line_of(const bfs_tune_key &k, const bfs_options &o, double best_us)
{
    int scale = 0;
    while (scale < 62 && (1LL << scale) < k.n) ++scale;
    const long long ef = k.n > 0 ? (long long)std::llround((double)k.nnz / (2.0 * (double)k.n)) : 0;
    char buf[1024];
    int m = std::snprintf(buf, sizeof buf,
                          "{\"scale\": %d, \"ef\": %lld, \"n\": %lld, \"nnz\": %lld, \"max_degree\": %lld, "
                          "\"isolated\": %lld, \"cus\": %d, \"mode\": %d",
                          scale, ef, (long long)k.n, (long long)k.nnz, (long long)k.max_degree,
                          (long long)k.isolated, k.cus, k.mode);
    std::string s(buf, (size_t)std::max(m, 0));
    for (const Field &f : kTuned) {
        m = std::snprintf(buf, sizeof buf, ", \"%s\": %d", f.name, o.*(f.member));
        s.append(buf, (size_t)std::max(m, 0));
    }
    m = std::snprintf(buf, sizeof buf, ", \"best_us\": %.3f}", best_us);
    s.append(buf, (size_t)std::max(m, 0));
    return s;
}

}  // namespace
}  // namespace hybfs

using namespace hybfs;

extern "C" {

int bfs_tune_key_get(bfs_graph_t gh, int32_t mode, bfs_tune_key *key)
{
    clear_error();
    if (!gh || !key) return set_error(BFS_E_INVALID, "NULL argument");
    if (mode < 0 || mode > 1) return set_error(BFS_E_INVALID, "mode must be 0 (single-root) or 1 (batched)");
    const Graph *g = reinterpret_cast<const Graph *>(gh);
    std::memset(key, 0, sizeof *key);
    key->n = g->n;
    key->nnz = g->nnz;
    key->max_degree = g->max_degree;
    key->isolated = g->isolated;
    key->cus = g->cus;
    key->mode = mode;
    return BFS_OK;
}

int bfs_tune_table_get(const char *path, const bfs_tune_key *key, bfs_options *opt, double *best_us)
{
    clear_error();
    if (!path || !key || !opt) return set_error(BFS_E_INVALID, "NULL argument");
    if (access(path, F_OK) != 0) {
        if (errno == ENOENT) return set_error(BFS_E_NOTFOUND, "no tune table at %s", path);
        return set_error(BFS_E_IO, "cannot reach the tune table %s: %s", path, std::strerror(errno));
    }
    std::ifstream in(path);
    if (!in.is_open()) return set_error(BFS_E_IO, "cannot read the tune table %s", path);
    bool hit = false;
    bfs_options best = *opt;
    double t_best = 0.0;
    std::string line;
    while (std::getline(in, line)) {
        if (!same_key(line, *key)) continue;
        bfs_options o;
        double t;
        if (line_options(line, *opt, &o, &t)) {   // the last valid entry counts
            best = o;
            t_best = t;
            hit = true;
        }
    }
    if (in.bad()) return set_error(BFS_E_IO, "error reading the tune table %s", path);
    if (!hit) return set_error(BFS_E_NOTFOUND, "no entry for this graph, device and mode in %s", path);
    *opt = best;
    if (best_us) *best_us = t_best;
    return BFS_OK;
}

int bfs_tune_table_put(const char *path, const bfs_tune_key *key, const bfs_options *opt, double best_us)
{
    clear_error();
    if (!path || !key || !opt) return set_error(BFS_E_INVALID, "NULL argument");
    if (key->mode < 0 || key->mode > 1) return set_error(BFS_E_INVALID, "mode must be 0 or 1");
    int rc = validate_options(*opt);
    if (rc) return rc;
    if (!std::isfinite(best_us) || best_us < 0) return set_error(BFS_E_INVALID, "best_us must be finite and >= 0");
    std::lock_guard<std::mutex> lk(g_table_mu);
    const FileLock flk(path);
    if (flk.fd < 0)
        return set_error(BFS_E_IO, "cannot lock the tune table %s.lock: %s", path, std::strerror(flk.err));
    std::vector<std::string> keep;
    if (access(path, F_OK) == 0) {
        std::ifstream in(path);
        if (!in.is_open()) return set_error(BFS_E_IO, "cannot read the tune table %s", path);
        std::string line;
        while (std::getline(in, line))
            if (!line.empty() && !same_key(line, *key)) keep.push_back(line);
        if (in.bad()) return set_error(BFS_E_IO, "error reading the tune table %s", path);
    } else if (errno != ENOENT) {
        return set_error(BFS_E_IO, "cannot reach the tune table %s: %s", path, std::strerror(errno));
    }
    keep.push_back(line_of(*key, *opt, best_us));
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out.is_open()) return set_error(BFS_E_IO, "cannot write %s: %s", tmp.c_str(), std::strerror(errno));
        for (const std::string &l : keep) out << l << '\n';
        out.flush();
        if (!out.good()) {
            std::remove(tmp.c_str());
            return set_error(BFS_E_IO, "error writing %s", tmp.c_str());
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        const int er = errno;
        std::remove(tmp.c_str());
        return set_error(BFS_E_IO, "cannot replace the tune table %s: %s", path, std::strerror(er));
    }
    return BFS_OK;
}

}  // extern "C"
