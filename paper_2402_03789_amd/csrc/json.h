// Minimal JSON reader for the weights-file header (objects, arrays, numbers,
// strings, true/false/null).  Throws std::runtime_error on malformed input.
#pragma once

#include <cstdlib>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace sn {

struct Json {
  enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
  bool b = false;
  double num = 0;
  std::string str;
  std::vector<Json> arr;
  std::map<std::string, Json> obj;

  const Json& at(const std::string& k) const {
    auto it = obj.find(k);
    if (kind != Obj || it == obj.end()) throw std::runtime_error("missing key: " + k);
    return it->second;
  }
  bool has(const std::string& k) const { return kind == Obj && obj.count(k); }
  double number() const {
    if (kind != Num) throw std::runtime_error("expected number");
    return num;
  }
  int integer() const { return (int)number(); }
  const std::string& string() const {
    if (kind != Str) throw std::runtime_error("expected string");
    return str;
  }
  const std::vector<Json>& array() const {
    if (kind != Arr) throw std::runtime_error("expected array");
    return arr;
  }
};

class JsonParser {
 public:
  explicit JsonParser(const std::string& s) : s_(s) {}
  Json parse() {
    Json v = value();
    ws();
    if (i_ != s_.size()) throw std::runtime_error("trailing characters in JSON");
    return v;
  }

 private:
  const std::string& s_;
  size_t i_ = 0;
  void ws() {
    while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\n' || s_[i_] == '\t' || s_[i_] == '\r')) ++i_;
  }
  char peek() {
    ws();
    if (i_ >= s_.size()) throw std::runtime_error("unexpected end of JSON");
    return s_[i_];
  }
  void expect(char c) {
    if (peek() != c) throw std::runtime_error(std::string("expected '") + c + "' in JSON");
    ++i_;
  }
  Json value() {
    char c = peek();
    Json v;
    if (c == '{') {
      v.kind = Json::Obj;
      ++i_;
      if (peek() == '}') { ++i_; return v; }
      while (true) {
        Json k = value();
        if (k.kind != Json::Str) throw std::runtime_error("object key must be a string");
        expect(':');
        v.obj[k.str] = value();
        if (peek() == ',') { ++i_; continue; }
        expect('}');
        return v;
      }
    }
    if (c == '[') {
      v.kind = Json::Arr;
      ++i_;
      if (peek() == ']') { ++i_; return v; }
      while (true) {
        v.arr.push_back(value());
        if (peek() == ',') { ++i_; continue; }
        expect(']');
        return v;
      }
    }
    if (c == '"') {
      v.kind = Json::Str;
      ++i_;
      while (i_ < s_.size() && s_[i_] != '"') {
        if (s_[i_] == '\\') {
          ++i_;
          if (i_ >= s_.size()) break;
          char e = s_[i_];
          v.str += (e == 'n') ? '\n' : (e == 't') ? '\t' : e;
        } else {
          v.str += s_[i_];
        }
        ++i_;
      }
      if (i_ >= s_.size()) throw std::runtime_error("unterminated string");
      ++i_;
      return v;
    }
    if (s_.compare(i_, 4, "true") == 0) { i_ += 4; v.kind = Json::Bool; v.b = true; return v; }
    if (s_.compare(i_, 5, "false") == 0) { i_ += 5; v.kind = Json::Bool; return v; }
    if (s_.compare(i_, 4, "null") == 0) { i_ += 4; return v; }
    const char* b = s_.c_str() + i_;
    char* e = nullptr;
    v.num = std::strtod(b, &e);
    if (e == b) throw std::runtime_error("bad JSON value");
    v.kind = Json::Num;
    i_ += (size_t)(e - b);
    return v;
  }
};

}  // namespace sn
