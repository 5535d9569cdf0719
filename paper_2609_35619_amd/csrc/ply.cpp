// Scene files: the binary little-endian PLY layout the 3DGS and 2DGS trainers
// write (Sec. II-A: a standard 3DGS scene is a set of Gaussians with mean,
// rotation quaternion, per-axis scale and opacity).  Per vertex: x y z,
// opacity (logit), scale_0 scale_1 [scale_2] (log; 2DGS files have two: the
// third axis is flat, scale 0), rot_0..rot_3 (w, x, y, z); every other vertex
// property (normals, spherical-harmonic colours) is skipped.  The parser
// returns activated parameters: linear scales exp(s) and opacities
// sigmoid(o), computed in double.  Host code only.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace {

int type_size(const std::string &t)
{
    if (t == "char" || t == "int8" || t == "uchar" || t == "uint8") return 1;
    if (t == "short" || t == "int16" || t == "ushort" || t == "uint16") return 2;
    if (t == "int" || t == "int32" || t == "uint" || t == "uint32" || t == "float" || t == "float32") return 4;
    if (t == "double" || t == "float64") return 8;
    return 0;
}

double read_as_double(const unsigned char *p, const std::string &t)
{
    if (t == "float" || t == "float32") {
        float v;
        std::memcpy(&v, p, 4);
        return v;
    }
    if (t == "double" || t == "float64") {
        double v;
        std::memcpy(&v, p, 8);
        return v;
    }
    if (t == "char" || t == "int8") return (double)*(const int8_t *)p;
    if (t == "uchar" || t == "uint8") return (double)*p;
    if (t == "short" || t == "int16") {
        int16_t v;
        std::memcpy(&v, p, 2);
        return v;
    }
    if (t == "ushort" || t == "uint16") {
        uint16_t v;
        std::memcpy(&v, p, 2);
        return v;
    }
    if (t == "int" || t == "int32") {
        int32_t v;
        std::memcpy(&v, p, 4);
        return v;
    }
    uint32_t v;
    std::memcpy(&v, p, 4);
    return v;
}

struct Prop {
    std::string type, name;
    int offset;
};

struct Element {
    std::string name;
    int64_t count = 0;
    std::vector<Prop> props;
    int stride = 0;
    bool has_list = false;
};

struct PlyFile {
    FILE *f = nullptr;
    ~PlyFile()
    {
        if (f) std::fclose(f);
    }
};

csplat_status err(const std::string &m) { return csplat::fail(CSPLAT_E_INVALID, m); }

// Reads the header; on success the file is positioned at the first data byte.
csplat_status read_header(FILE *f, std::vector<Element> &els)
{
    char line[1024];
    if (!std::fgets(line, sizeof line, f) || std::strncmp(line, "ply", 3) != 0) return err("ply: not a PLY file");
    bool format_ok = false;
    for (;;) {
        if (!std::fgets(line, sizeof line, f)) return err("ply: truncated header");
        std::string s(line);
        while (!s.empty() && (s.back() == '\n' || s.back() == '\r')) s.pop_back();
        if (s == "end_header") break;
        char a[256], b[256], c[256];
        if (std::sscanf(s.c_str(), "format %255s %255s", a, b) == 2) {
            if (std::string(a) != "binary_little_endian")
                return err("ply: only binary_little_endian files are supported (found " + std::string(a) + ")");
            format_ok = true;
        } else if (std::sscanf(s.c_str(), "element %255s %255s", a, b) == 2) {
            Element e;
            e.name = a;
            char *end = nullptr;
            e.count = std::strtoll(b, &end, 10);
            if (!end || *end || e.count < 0) return err("ply: bad element count");
            els.push_back(e);
        } else if (std::sscanf(s.c_str(), "property list %255s %255s %255s", a, b, c) == 3) {
            if (els.empty()) return err("ply: property before element");
            els.back().has_list = true;
        } else if (std::sscanf(s.c_str(), "property %255s %255s", a, b) == 2) {
            if (els.empty()) return err("ply: property before element");
            const int sz = type_size(a);
            if (!sz) return err("ply: unknown property type " + std::string(a));
            Element &e = els.back();
            e.props.push_back(Prop{a, b, e.stride});
            e.stride += sz;
        }
        // comment / obj_info lines are ignored
    }
    if (!format_ok) return err("ply: missing format line");
    return CSPLAT_OK;
}

}  // namespace

extern "C" csplat_status csplat_ply_read(const char *path, int64_t capacity, int64_t *n, float *means, float *quats,
                                         float *scales, float *opacity)
{
    if (!path || !n) return err("ply_read: NULL argument");
    PlyFile pf;
    pf.f = std::fopen(path, "rb");
    if (!pf.f) return err(std::string("ply_read: cannot open ") + path);
    std::vector<Element> els;
    csplat_status s = read_header(pf.f, els);
    if (s != CSPLAT_OK) return s;
    // elements before "vertex" must be skippable (fixed-size records)
    int64_t skip = 0;
    const Element *v = nullptr;
    for (const Element &e : els) {
        if (e.name == "vertex") {
            v = &e;
            break;
        }
        if (e.has_list && e.count > 0) return err("ply_read: a list element precedes the vertices");
        skip += e.count * e.stride;
    }
    if (!v) return err("ply_read: no vertex element");
    if (v->has_list) return err("ply_read: list properties in the vertex element");
    const char *need[] = {"x", "y", "z", "opacity", "scale_0", "scale_1", "rot_0", "rot_1", "rot_2", "rot_3"};
    const Prop *idx[11] = {nullptr};
    for (int k = 0; k < 10; ++k)
        for (const Prop &p : v->props)
            if (p.name == need[k]) idx[k] = &p;
    for (const Prop &p : v->props)
        if (p.name == "scale_2") idx[10] = &p;
    for (int k = 0; k < 10; ++k)
        if (!idx[k]) return err(std::string("ply_read: vertex property missing: ") + need[k]);
    *n = v->count;
    if (v->count == 0) return CSPLAT_OK;
    if (capacity < v->count) return capacity == 0 ? CSPLAT_OK : err("ply_read: capacity below the vertex count");
    if (!means || !quats || !scales || !opacity) return err("ply_read: NULL output array");
    if (skip && std::fseek(pf.f, (long)skip, SEEK_CUR) != 0) return err("ply_read: truncated file");
    std::vector<unsigned char> buf((size_t)v->stride * 4096);
    for (int64_t i0 = 0; i0 < v->count; i0 += 4096) {
        const int64_t cnt = std::min<int64_t>(4096, v->count - i0);
        if (std::fread(buf.data(), (size_t)v->stride, (size_t)cnt, pf.f) != (size_t)cnt)
            return err("ply_read: truncated vertex data");
        for (int64_t k = 0; k < cnt; ++k) {
            const unsigned char *r = buf.data() + (size_t)k * v->stride;
            auto val = [&](int j) { return read_as_double(r + idx[j]->offset, idx[j]->type); };
            const int64_t i = i0 + k;
            means[3 * i] = (float)val(0);
            means[3 * i + 1] = (float)val(1);
            means[3 * i + 2] = (float)val(2);
            opacity[i] = (float)(1.0 / (1.0 + std::exp(-val(3))));
            scales[3 * i] = (float)std::exp(val(4));
            scales[3 * i + 1] = (float)std::exp(val(5));
            scales[3 * i + 2] = idx[10] ? (float)std::exp(val(10)) : 0.f;
            for (int c = 0; c < 4; ++c) quats[4 * i + c] = (float)val(6 + c);
        }
    }
    return CSPLAT_OK;
}

extern "C" csplat_status csplat_scene_load_ply(csplat_ctx *ctx, const char *path, const csplat_scene_opts *opts,
                                               csplat_scene **out)
{
    if (!ctx || !path || !out) return err("scene_load_ply: NULL argument");
    int64_t n = 0;
    csplat_status s = csplat_ply_read(path, 0, &n, nullptr, nullptr, nullptr, nullptr);
    if (s != CSPLAT_OK) return s;
    std::vector<float> means((size_t)n * 3), quats((size_t)n * 4), scales((size_t)n * 3), opacity((size_t)n);
    s = csplat_ply_read(path, n, &n, means.data(), quats.data(), scales.data(), opacity.data());
    if (s != CSPLAT_OK) return s;
    csplat_scene_opts o{};
    if (opts) o = *opts;
    o.param_mode = CSPLAT_PARAM_ACTIVATED;
    return csplat_scene_load(ctx, n, means.data(), quats.data(), scales.data(), opacity.data(), &o, out);
}
