// Errors, hashing, files, configuration helpers and flat JSON lines.
#include <dlfcn.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cctype>
#include <cerrno>
#include <functional>
#include <thread>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "internal.h"

namespace conv2d {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg)
{
    g_last_error = msg;
    return status;
}

void clear_error() { g_last_error.clear(); }

const char* last_error_cstr() { return g_last_error.c_str(); }

int hip_fail(hipError_t e, const char* what)
{
    return fail(CONV2D_EHIP, std::string(what) + ": " + hipGetErrorName(e) + " (" +
                                 hipGetErrorString(e) + ")");
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h)
{
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t fnv1a(const std::string& s, uint64_t h) { return fnv1a(s.data(), s.size(), h); }

std::string code_text(const std::string& s)
{
    std::string out;
    out.reserve(s.size());
    const size_t n = s.size();
    auto space = [&] {
        if (!out.empty() && out.back() != ' ' && out.back() != '\n') out += ' ';
    };
    size_t i = 0;
    while (i < n) {
        const char c = s[i];
        if (c == '/' && i + 1 < n && s[i + 1] == '/') {           // line comment: up to the newline
            while (i < n && s[i] != '\n') ++i;
        } else if (c == '/' && i + 1 < n && s[i + 1] == '*') {    // block comment: one space
            const size_t e = s.find("*/", i + 2);
            i = e == std::string::npos ? n : e + 2;
            space();
        } else if (c == '"' || c == '\'') {                       // literal, copied as is
            out += c;
            ++i;
            while (i < n && s[i] != c) {
                if (s[i] == '\\' && i + 1 < n) out += s[i++];
                out += s[i++];
            }
            if (i < n) out += s[i++];
        } else if (c == '\n') {                                   // newlines matter (directives)
            while (!out.empty() && out.back() == ' ') out.pop_back();
            if (!out.empty() && out.back() != '\n') out += '\n';
            ++i;
        } else if (c == ' ' || c == '\t' || c == '\r' || c == '\f' || c == '\v') {
            space();
            ++i;
        } else {
            out += c;
            ++i;
        }
    }
    while (!out.empty() && (out.back() == ' ' || out.back() == '\n')) out.pop_back();
    return out;
}

std::string hex64(uint64_t v)
{
    char b[17];
    std::snprintf(b, sizeof b, "%016llx", (unsigned long long)v);
    return b;
}

std::string env_str(const char* name, const char* dflt)
{
    const char* v = std::getenv(name);
    return (v && *v) ? std::string(v) : std::string(dflt);
}

std::string library_dir()
{
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&library_dir), &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        size_t k = p.find_last_of('/');
        return k == std::string::npos ? std::string(".") : p.substr(0, k);
    }
    return ".";
}

bool make_dirs(const std::string& path)
{
    if (path.empty()) return false;
    std::string cur;
    std::stringstream ss(path);
    std::string part;
    if (path[0] == '/') cur = "/";
    while (std::getline(ss, part, '/')) {
        if (part.empty()) continue;
        cur += part + "/";
        if (mkdir(cur.c_str(), 0775) != 0 && errno != EEXIST) return false;
    }
    return true;
}

bool write_file_atomic(const std::string& path, const void* data, size_t n)
{
    std::string tmp = path + ".tmp" + std::to_string(getpid()) + "_" +
                      std::to_string(std::hash<std::thread::id>{}(std::this_thread::get_id()));
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    bool ok = std::fwrite(data, 1, n, f) == n;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

bool read_file(const std::string& path, std::vector<char>& out)
{
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    out.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return true;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- configs

static bool in_set(int v, std::initializer_list<int> s)
{
    for (int x : s)
        if (x == v) return true;
    return false;
}

bool config_axes_valid(const conv2d_config& c, std::string* why)
{
    auto bad = [&](const char* m) { if (why) *why = m; return false; };
    if (!in_set(c.block_x, {16, 32, 64, 128})) return bad("block_x must be 16, 32, 64 or 128");
    if (!in_set(c.block_y, {1, 2, 4, 8, 16})) return bad("block_y must be 1, 2, 4, 8 or 16");
    if (!in_set(c.tile_x, {1, 2, 4, 8})) return bad("tile_x must be 1, 2, 4 or 8");
    if (!in_set(c.tile_y, {1, 2, 4, 8})) return bad("tile_y must be 1, 2, 4 or 8");
    if (!in_set(c.use_lds, {0, 1})) return bad("use_lds must be 0 or 1");
    if (!in_set(c.filter_in_const, {0, 1})) return bad("filter_in_const must be 0 or 1");
    if (!in_set(c.unroll, {0, 1, 2, 4})) return bad("unroll must be 0 (full), 1, 2 or 4");
    if (c.block_x * c.block_y > kMaxThreads) return bad("block_x * block_y exceeds 1024 threads");
    return true;
}

std::string config_str(const conv2d_config& c)
{
    char b[96];
    std::snprintf(b, sizeof b, "%d,%d,%d,%d,%d,%d,%d", c.block_x, c.block_y, c.tile_x, c.tile_y,
                  c.use_lds, c.filter_in_const, c.unroll);
    return b;
}

bool parse_config(const std::string& s, conv2d_config* c)
{
    conv2d_config t{};
    int n = std::sscanf(s.c_str(), "%d,%d,%d,%d,%d,%d,%d", &t.block_x, &t.block_y, &t.tile_x,
                        &t.tile_y, &t.use_lds, &t.filter_in_const, &t.unroll);
    if (n == 6) t.unroll = 1;
    else if (n != 7) return false;
    *c = t;
    return true;
}

static int key_at(const conv2d_config& c, int k)
{
    switch (k) {
    case 0: return c.block_x;
    case 1: return c.block_y;
    case 2: return c.tile_x;
    case 3: return c.tile_y;
    case 4: return c.use_lds;
    case 5: return c.filter_in_const;
    default: return c.unroll;
    }
}

bool config_less(const conv2d_config& a, const conv2d_config& b)
{
    for (int k = 0; k < 7; ++k)
        if (key_at(a, k) != key_at(b, k)) return key_at(a, k) < key_at(b, k);
    return false;
}

bool config_equal(const conv2d_config& a, const conv2d_config& b)
{
    return !config_less(a, b) && !config_less(b, a);
}

// Mirrors the LDS tile layout of the kernel: rows = by*ty + fh - 1, a padded
// pitch of whole input-vector chunks rounded to 4 floats (+4 when it is a
// multiple of 32), for the widest input vector the kernel may be built with.
int lds_bytes(int fh, int fw, const conv2d_config& c)
{
    if (!c.use_lds) return 0;
    const int rows = c.block_y * c.tile_y + fh - 1;
    const int cols = c.block_x * c.tile_x + fw - 1;
    int best = 0;
    for (int vin : {1, 2, 4}) {
        int chunks = (cols + vin - 1) / vin;
        int pitch = ((chunks * vin + 3) / 4) * 4;
        if (pitch % 32 == 0) pitch += 4;
        best = std::max(best, rows * pitch * 4);
    }
    return best;
}

int shape_check(const conv2d_shape& s)
{
    if (s.out_h < 1 || s.out_w < 1)
        return fail(CONV2D_EINVAL, "out_h and out_w must be >= 1");
    if (s.filt_h < 1 || s.filt_w < 1 || s.filt_h > kMaxFilter || s.filt_w > kMaxFilter)
        return fail(CONV2D_EINVAL, "filter sizes must be in 1..63");
    if ((long long)s.out_w + s.filt_w - 1 > (1ll << 28) || (long long)s.out_h + s.filt_h - 1 > (1ll << 28))
        return fail(CONV2D_EINVAL, "image side too large");
    return CONV2D_OK;
}

// ---------------------------------------------------------------- JSON lines

std::string json_escape(const std::string& s)
{
    std::string o;
    for (char ch : s) {
        if (ch == '"' || ch == '\\') { o += '\\'; o += ch; }
        else if (ch == '\n') o += "\\n";
        else if ((unsigned char)ch < 0x20) o += ' ';
        else o += ch;
    }
    return o;
}

namespace {
struct Cursor {
    const std::string& s;
    size_t i = 0;
    void ws() { while (i < s.size() && std::isspace((unsigned char)s[i])) ++i; }
    bool eat(char c) { ws(); if (i < s.size() && s[i] == c) { ++i; return true; } return false; }
    bool str(std::string* out)
    {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        ++i;
        std::string o;
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\' && i + 1 < s.size()) { ++i; o += (s[i] == 'n') ? '\n' : s[i]; }
            else o += s[i];
            ++i;
        }
        if (i >= s.size()) return false;
        ++i;
        *out = o;
        return true;
    }
    bool num(double* out)
    {
        ws();
        const char* b = s.c_str() + i;
        char* e = nullptr;
        double v = std::strtod(b, &e);
        if (e == b) {
            if (s.compare(i, 4, "null") == 0) { i += 4; *out = 0.0; return true; }
            if (s.compare(i, 4, "true") == 0) { i += 4; *out = 1.0; return true; }
            if (s.compare(i, 5, "false") == 0) { i += 5; *out = 0.0; return true; }
            return false;
        }
        i += (size_t)(e - b);
        *out = v;
        return true;
    }
};
}  // namespace

bool json_parse_line(const std::string& line, JsonObj* out)
{
    Cursor c{line};
    if (!c.eat('{')) return false;
    if (c.eat('}')) return true;
    for (;;) {
        std::string key;
        if (!c.str(&key) || !c.eat(':')) return false;
        c.ws();
        if (c.i < line.size() && line[c.i] == '"') {
            std::string v;
            if (!c.str(&v)) return false;
            out->str[key] = v;
        } else if (c.eat('[')) {
            std::vector<double> a;
            if (!c.eat(']')) {
                for (;;) {
                    double v;
                    if (!c.num(&v)) return false;
                    a.push_back(v);
                    if (c.eat(']')) break;
                    if (!c.eat(',')) return false;
                }
            }
            out->arr[key] = a;
        } else {
            double v;
            if (!c.num(&v)) return false;
            out->num[key] = v;
        }
        if (c.eat('}')) return true;
        if (!c.eat(',')) return false;
    }
}

bool append_line(const std::string& path, const std::string& line)
{
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return false;
    bool ok = std::fprintf(f, "%s\n", line.c_str()) > 0;
    return (std::fclose(f) == 0) && ok;
}

}  // namespace conv2d
